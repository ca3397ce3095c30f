"""Shared helpers of the GPU parity tests (imports torch and the library lazily)."""

import numpy as np
import pytest

import oracle


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1309_7473_amd as mm  # noqa: F401  (fails loudly if libmm.so is missing)
    return mm


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def relmax(a, b):
    """Element-wise gate: max |a - b| over max |b|.  A relative L2 error can
    hide a large error confined to a few entries; this cannot."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    mb = np.abs(b).max() if b.size else 0.0
    return np.abs(a - b).max() / (mb if mb > 0 else 1.0) if a.size else 0.0


class Pair:
    """The same seeded inputs seen by the oracle and by the GPU library."""

    def __init__(self, inp, tod_dtype="f32", **kw):
        mm = need_gpu()
        import torch
        self.inp = inp
        self.torch = torch
        self.o = oracle.OracleScan(inp)
        self.B = oracle.binned_blocks(self.o, oracle.detector_weights(self.o))
        self.Bj = oracle.binned_blocks(self.o, np.ones(self.o.ndet))
        self.mask = oracle.active_mask(self.o, self.B, kw.get("mask_rcond", 0) or 1e-3)
        self.g = mm.Scan(inp, tod_dtype=tod_dtype, **kw)
        self.nc, self.npix = inp.ncomp, inp.ny * inp.nx

    def dev(self, a):
        return self.torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()

    def host(self, t):
        self.torch.cuda.synchronize()
        return t.cpu().numpy()

    def A_oracle(self, x):
        return oracle.apply_A(self.o, x, self.mask)

    def A_gpu(self, x):
        return self.host(self.g.apply_A(self.dev(x)))

    def masked_random(self, seed=0):
        r = np.random.default_rng(seed).standard_normal((self.nc, self.npix))
        return (r * self.mask).ravel()

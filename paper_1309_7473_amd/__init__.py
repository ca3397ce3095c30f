"""MI355X map-making library: Python binding of libmm.so (include/mm.h).

The functions here have the C ABI's names and only marshal arguments
(torch device tensors -> pointers, the current HIP stream); every step of the
computation runs in the HIP kernels of libmm.so.  Importing the package fails
if libmm.so has not been built.

`Scan` keeps the device copies of one scan's inputs and its workspace alive
for the lifetime of a handle.
"""

import ctypes as C

import numpy as np
import torch

from ._abi import (  # noqa: F401
    lib, check, MMError, mm_scan_desc, mm_precon_opts, mm_pcg_opts, mm_pcg_result,
    mm_scan_info, MM_OK, MM_ENOCONV, MM_EINVAL, MM_ENOMEM, MM_EDEVICE, MM_ENOTBUILT,
    MM_EBREAKDOWN, MM_F32, MM_BF16, MM_F64, MM_M_NONE, MM_M_JACOBI, MM_M_BINNED,
    MM_M_CIRCULANT, MM_M_LEARNED, MM_M_TILED, LIB_PATH, mm_profile, PROFILE_STAGES, MM_SCATTER_AUTO,
    MM_SCATTER_ATOMIC, MM_SCATTER_SAMPLES, mm_train_opts, MM_ACC_F64, MM_ACC_F32X2, MM_POINT_STORED,
    MM_POINT_BORESIGHT, MM_PTC_AUTO, MM_PTC_OFF,
)

PRECON = {"none": MM_M_NONE, "jacobi": MM_M_JACOBI, "binned": MM_M_BINNED,
          "circulant": MM_M_CIRCULANT, "learned": MM_M_LEARNED, "tiled": MM_M_TILED}


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _ptr(t, dtype=None, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


# ------------------------------------------------------------- raw ABI calls
def mm_scan_workspace_bytes(desc):
    return int(lib.mm_scan_workspace_bytes(C.byref(desc)))


def mm_create_scan(desc, stream=None):
    h = C.c_void_p()
    check(lib.mm_create_scan(C.byref(desc), _stream(stream), C.byref(h)), "mm_create_scan")
    return h


def mm_destroy_scan(h):
    lib.mm_destroy_scan(h)


def mm_rhs(h, tod, b, stream=None):
    check(lib.mm_rhs(h, _ptr(tod, name="tod"), _ptr(b, torch.float64, name="b"), _stream(stream)),
          "mm_rhs")


def mm_apply_A(h, x, y, stream=None):
    check(lib.mm_apply_A(h, _ptr(x, torch.float64, name="x"), _ptr(y, torch.float64, name="y"),
                         _stream(stream)), "mm_apply_A")


def mm_build_precon(h, precon, opts=None, stream=None):
    o = None if opts is None else C.byref(opts)
    check(lib.mm_build_precon(h, int(precon), o, _stream(stream)), "mm_build_precon")


def mm_apply_precon_binned(h, precon, r, z, stream=None):
    check(lib.mm_apply_precon_binned(h, int(precon), _ptr(r, torch.float64, name="r"),
                                     _ptr(z, torch.float64, name="z"), _stream(stream)),
          "mm_apply_precon_binned")


def mm_apply_precon_circulant(h, r, z, stream=None):
    check(lib.mm_apply_precon_circulant(h, _ptr(r, torch.float64, name="r"),
                                        _ptr(z, torch.float64, name="z"), _stream(stream)),
          "mm_apply_precon_circulant")


def mm_tiled_workspace_bytes(h, tile):
    return int(lib.mm_tiled_workspace_bytes(h, int(tile)))


def mm_apply_precon_tiled(h, r, z, stream=None):
    check(lib.mm_apply_precon_tiled(h, _ptr(r, torch.float64, name="r"),
                                    _ptr(z, torch.float64, name="z"), _stream(stream)),
          "mm_apply_precon_tiled")


def _pcg_opts(tol, maxiter, check_every=1, x0=False, graph=False, flexible=False, refine=0,
              true_residual=False):
    o = mm_pcg_opts()
    o.tol, o.maxiter, o.check_every, o.use_x0 = float(tol), int(maxiter), int(check_every), int(x0)
    o.graph = 1 if graph else 0
    o.flexible = 1 if flexible else 0
    o.refine = int(refine)
    o.true_residual = 1 if true_residual else 0
    return o


def mm_pcg_solve(h, precon, b, x, opts, stream=None, history_len=0):
    """Returns (status, result dict).  MM_ENOCONV is returned, not raised."""
    res = mm_pcg_result()
    hist = alpha = rho = None
    if history_len:
        hist = (C.c_double * (history_len + 1))()
        alpha = (C.c_double * history_len)()
        rho = (C.c_double * history_len)()
        res.history = C.cast(hist, C.POINTER(C.c_double))
        res.alpha = C.cast(alpha, C.POINTER(C.c_double))
        res.rho = C.cast(rho, C.POINTER(C.c_double))
    st = lib.mm_pcg_solve(h, int(precon), _ptr(b, torch.float64, name="b"),
                          _ptr(x, torch.float64, name="x"), C.byref(opts), C.byref(res),
                          _stream(stream))
    if st not in (MM_OK, MM_ENOCONV, MM_EBREAKDOWN):
        check(st, "mm_pcg_solve")
    out = _result_dict(res, st)
    if history_len:
        n = min(res.iters, history_len)
        out["history"] = np.array(hist[: n + 1])
        out["alpha"] = np.array(alpha[:n])
        out["rho"] = np.array(rho[:n])
    return st, out


def mm_pcg_solve_batch(handles, precon, bs, xs, opts, stream=None):
    """Independent solves of several scans.  Returns (status, [result dict])."""
    n = len(handles)
    if not (len(bs) == len(xs) == n) or n < 1:
        raise ValueError("handles, bs and xs must have the same non-zero length")
    H = (C.c_void_p * n)(*[C.c_void_p(h.value if isinstance(h, C.c_void_p) else h) for h in handles])
    B = (C.c_void_p * n)(*[_ptr(b, torch.float64, name="b") for b in bs])
    X = (C.c_void_p * n)(*[_ptr(x, torch.float64, name="x") for x in xs])
    res = (mm_pcg_result * n)()
    sts = (C.c_int32 * n)()
    st = lib.mm_pcg_solve_batch(H, n, int(precon), B, X, C.byref(opts), res, sts, _stream(stream))
    if st not in (MM_OK, MM_ENOCONV, MM_EBREAKDOWN):
        check(st, "mm_pcg_solve_batch")
    out = [_result_dict(res[i], int(sts[i])) for i in range(n)]
    return st, out


def mm_precon_judge(h, candidates, b, x, opts, stream=None):
    """Solves A x = b with each candidate preconditioner (names or enums);
    returns (status, chosen enum, [result dict])."""
    cand = [PRECON[c] if isinstance(c, str) else int(c) for c in candidates]
    n = len(cand)
    ca = (C.c_int32 * n)(*cand)
    res = (mm_pcg_result * n)()
    chosen = C.c_int32(-1)
    st = lib.mm_precon_judge(h, ca, n, _ptr(b, torch.float64, name="b"),
                             _ptr(x, torch.float64, name="x"), C.byref(opts), res,
                             C.byref(chosen), _stream(stream))
    if st not in (MM_OK, MM_ENOCONV, MM_EBREAKDOWN):
        check(st, "mm_precon_judge")
    return st, int(chosen.value), [_result_dict(res[i], None) for i in range(n)]


def _result_dict(res, st):
    return dict(status=st, iters=res.iters, converged=bool(res.converged),
                rel_resid=res.rel_resid, t_solve_s=res.t_solve_s, t_setup_s=res.t_setup_s,
                true_rel_resid=res.true_rel_resid, restarts=res.restarts)


def mm_map_spectra(h, x, pixel_arcmin, dell, nbins, ncomp, stream=None):
    """Binned TT (and EE, BB) spectra of a device map: (spectra (1 or 3, nbins),
    counts (nbins,))."""
    nout = 3 if ncomp == 3 else 1
    spec = np.zeros((nout, int(nbins)), np.float64)
    cnt = np.zeros(int(nbins), np.float64)
    check(lib.mm_map_spectra(h, _ptr(x, torch.float64, name="x"), float(pixel_arcmin), float(dell),
                             int(nbins), spec.ctypes.data_as(C.c_void_p),
                             cnt.ctypes.data_as(C.c_void_p), _stream(stream)), "mm_map_spectra")
    return spec, cnt


def mm_map_spectra_noalloc(h, x, pixel_arcmin, dell, nbins, ncomp, stream=None):
    """mm_map_spectra with its scratch in the library's static device array
    (no device memory from the caller or the scan's workspace)."""
    nout = 3 if ncomp == 3 else 1
    spec = np.zeros((nout, int(nbins)), np.float64)
    cnt = np.zeros(int(nbins), np.float64)
    check(lib.mm_map_spectra_noalloc(h, _ptr(x, torch.float64, name="x"), float(pixel_arcmin),
                                     float(dell), int(nbins), spec.ctypes.data_as(C.c_void_p),
                                     cnt.ctypes.data_as(C.c_void_p), _stream(stream)),
          "mm_map_spectra_noalloc")
    return spec, cnt


def mm_anorm_error_estimate(alpha, rho, delay=4):
    """Delayed A-norm error estimate from recorded PCG scalars (host)."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    r = np.ascontiguousarray(rho, dtype=np.float64)
    n = min(len(a), len(r))
    est = np.zeros(max(n - int(delay) + 1, 0), np.float64)
    check(lib.mm_anorm_error_estimate(a.ctypes.data_as(C.c_void_p), r.ctypes.data_as(C.c_void_p),
                                      int(n), int(delay), est.ctypes.data_as(C.c_void_p)),
          "mm_anorm_error_estimate")
    return est


def mm_spectrum_cv_error(c_iter, c_input, counts):
    """Per-bin spectrum error in cosmic-variance units (host, libmm)."""
    ci = np.ascontiguousarray(c_iter, dtype=np.float64)
    cn = np.ascontiguousarray(np.broadcast_to(c_input, ci.shape), dtype=np.float64)
    cnt = np.ascontiguousarray(counts, dtype=np.float64)
    nb = cnt.size
    if ci.size % nb:
        raise ValueError("c_iter must be [ncomp][nbins]")
    err = np.empty(ci.shape, np.float64)
    check(lib.mm_spectrum_cv_error(ci.ctypes.data_as(C.c_void_p), cn.ctypes.data_as(C.c_void_p),
                                   cnt.ctypes.data_as(C.c_void_p), ci.size // nb, nb,
                                   err.ctypes.data_as(C.c_void_p)), "mm_spectrum_cv_error")
    return err


def mm_cv_crossing_step(steps, errors, threshold=0.1, block=50):
    """CG step at which block-averaged errors first reach threshold, or None."""
    st = np.ascontiguousarray(steps, dtype=np.float64)
    er = np.ascontiguousarray(errors, dtype=np.float64)
    out = C.c_double(0.0)
    found = C.c_int32(0)
    check(lib.mm_cv_crossing_step(st.ctypes.data_as(C.c_void_p), er.ctypes.data_as(C.c_void_p),
                                  min(st.size, er.size), float(threshold), int(block),
                                  C.byref(out), C.byref(found)), "mm_cv_crossing_step")
    return float(out.value) if found.value else None


def mm_get_info(h):
    info = mm_scan_info()
    check(lib.mm_get_info(h, C.byref(info)), "mm_get_info")
    return {k: getattr(info, k) for k, _ in mm_scan_info._fields_}


def mm_get_mask(h, dst, stream=None):
    check(lib.mm_get_mask(h, _ptr(dst, torch.int32, name="dst"), _stream(stream)), "mm_get_mask")


def mm_profile_enable(h, enable=True):
    check(lib.mm_profile_enable(h, 1 if enable else 0), "mm_profile_enable")


def mm_profile_stages(h, stages=None):
    """Time only the named stages (PROFILE_STAGES names); None: every stage."""
    mask = 0xFFFFFFFF if stages is None else sum(1 << PROFILE_STAGES.index(n) for n in stages)
    check(lib.mm_profile_stages(h, mask), "mm_profile_stages")


def mm_profile_read(h):
    """Synchronises the timed launches; returns {stage: (ms, launches, samples)}."""
    p = mm_profile()
    check(lib.mm_profile_read(h, C.byref(p)), "mm_profile_read")
    return {PROFILE_STAGES[i]: (p.ms[i], p.launches[i], p.samples[i])
            for i in range(p.n_stages) if PROFILE_STAGES[i] and p.launches[i]}


def mm_learned_workspace_bytes(ncomp, ny, nx, batch):
    return int(lib.mm_learned_workspace_bytes(ncomp, ny, nx, batch))


def _host_f32(a, n, name):
    a = np.ascontiguousarray(a, dtype=np.float32).ravel()
    if a.size != n:
        raise ValueError(f"{name} must have {n} elements")
    return a


def mm_learned_create(ncomp, ny, nx, batch, workspace, w1, w2, stream=None):
    w1 = _host_f32(w1, 16 * ncomp * 25, "w1")
    w2 = _host_f32(w2, 16 * 16 * 25, "w2")
    h = C.c_void_p()
    check(lib.mm_learned_create(ncomp, ny, nx, batch, _ptr(workspace, torch.uint8, name="workspace"),
                                workspace.numel(), w1.ctypes.data_as(C.c_void_p),
                                w2.ctypes.data_as(C.c_void_p), _stream(stream), C.byref(h)),
          "mm_learned_create")
    return h


def mm_learned_destroy(h):
    lib.mm_learned_destroy(h)


def mm_learned_get(h, ncomp):
    w1 = np.empty(16 * ncomp * 25, np.float32)
    w2 = np.empty(16 * 16 * 25, np.float32)
    check(lib.mm_learned_get(h, w1.ctypes.data_as(C.c_void_p), w2.ctypes.data_as(C.c_void_p)),
          "mm_learned_get")
    return w1.reshape(16, ncomp, 5, 5), w2.reshape(16, 16, 5, 5)


def mm_learned_attach(scan_h, h):
    check(lib.mm_learned_attach(scan_h, h), "mm_learned_attach")


def mm_learned_make_pair(scan_h, x_f, x_k, r_w, t, e2, stream=None):
    check(lib.mm_learned_make_pair(scan_h, _ptr(x_f, torch.float64, name="x_f"),
                                   _ptr(x_k, torch.float64, name="x_k"),
                                   _ptr(r_w, torch.float32, name="r_w"),
                                   _ptr(t, torch.float32, name="t"), _ptr(e2, torch.float32, name="e2"),
                                   _stream(stream)), "mm_learned_make_pair")


def mm_learned_train(h, r_w, t, e2, npairs, opts, stream=None):
    hist = (C.c_double * max(1, opts.epochs))()
    check(lib.mm_learned_train(h, _ptr(r_w, torch.float32, name="r_w"),
                               _ptr(t, torch.float32, name="t"), _ptr(e2, torch.float32, name="e2"),
                               int(npairs), C.byref(opts), C.cast(hist, C.c_void_p), _stream(stream)),
          "mm_learned_train")
    return np.array(hist[: opts.epochs])


def mm_learned_loss(h, r_w, t, e2, npairs, stream=None):
    out = C.c_double()
    check(lib.mm_learned_loss(h, _ptr(r_w, torch.float32, name="r_w"),
                              _ptr(t, torch.float32, name="t"), _ptr(e2, torch.float32, name="e2"),
                              int(npairs), C.byref(out), _stream(stream)), "mm_learned_loss")
    return out.value


def mm_learned_forward(h, x, B, y, a1=None, a2=None, a3=None, stream=None):
    check(lib.mm_learned_forward(h, _ptr(x, torch.float32, name="x"), int(B),
                                 _ptr(y, torch.float32, name="y"), _ptr(a1), _ptr(a2), _ptr(a3),
                                 _stream(stream)), "mm_learned_forward")


def mm_learned_grad(h, r_w, t, e2, B, ncomp, stream=None):
    loss = C.c_double()
    g1 = np.empty(16 * ncomp * 25, np.float32)
    g2 = np.empty(16 * 16 * 25, np.float32)
    check(lib.mm_learned_grad(h, _ptr(r_w, torch.float32, name="r_w"),
                              _ptr(t, torch.float32, name="t"), _ptr(e2, torch.float32, name="e2"),
                              int(B), C.byref(loss), g1.ctypes.data_as(C.c_void_p),
                              g2.ctypes.data_as(C.c_void_p), _stream(stream)), "mm_learned_grad")
    return loss.value, g1.reshape(16, ncomp, 5, 5), g2.reshape(16, 16, 5, 5)


def mm_apply_precon_learned(h, r, z, stream=None):
    check(lib.mm_apply_precon_learned(h, _ptr(r, torch.float64, name="r"),
                                      _ptr(z, torch.float64, name="z"), _stream(stream)),
          "mm_apply_precon_learned")


def mm_last_error():
    return lib.mm_last_error().decode(errors="replace")


# ---------------------------------------------------------------- Scan owner
class Scan:
    """Device copies of one scan's inputs, its workspace and its handle.

    inputs: an object with ncomp, ny, nx, ndet (pix.shape[0]), nsamp, fsample,
    pix (int32 [ndet][nsamp]), cos2psi/sin2psi (float32 or None) and
    inv_noise (float32 [ndet][nsamp/2+1]) as numpy arrays or device tensors.
    """

    def __init__(self, inputs, tod_dtype="f32", det_group=0, fft_m1=0, fft_cols=0,
                 mask_rcond=0.0, scatter="auto", acc="f64", pointing="auto", device="cuda",
                 stream=None, pointing_code="auto"):
        """pointing: "stored" (inputs.pix, cos2psi, sin2psi), "boresight"
        (inputs.bore [6][nsamp] and inputs.det_off [4][ndet], float64: each
        sample's pointing is computed on the GPU when it is needed), or "auto"
        (stored when inputs.pix is given).  pointing_code: "auto" lets pass 1
        read a chunk-coded copy of stored pointing when every chunk fits,
        "off" keeps the stored pixels and time-major angles."""
        self.device = torch.device(device)
        dev = self.device

        def up(a, dt):
            if a is None:
                return None
            if isinstance(a, torch.Tensor):
                return a.to(device=dev, dtype=dt).contiguous()
            return torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dt)

        if pointing == "auto":
            pointing = "stored" if getattr(inputs, "pix", None) is not None else "boresight"
        if pointing not in ("stored", "boresight"):
            raise ValueError(f"unknown pointing {pointing!r}")
        self.pointing = pointing
        self.ncomp, self.ny, self.nx = int(inputs.ncomp), int(inputs.ny), int(inputs.nx)
        self.inv_noise = up(inputs.inv_noise, torch.float32)
        if pointing == "stored":
            self.pix = up(inputs.pix, torch.int32)
            self.cos2psi = up(inputs.cos2psi, torch.float32)
            self.sin2psi = up(inputs.sin2psi, torch.float32)
            self.bore = self.det_off = None
            self.ndet, self.nsamp = int(self.pix.shape[0]), int(self.pix.shape[1])
        else:
            self.pix = self.cos2psi = self.sin2psi = None
            self.bore = up(inputs.bore, torch.float64)
            self.det_off = up(inputs.det_off, torch.float64)
            if self.bore.dim() != 2 or self.bore.shape[0] != 6:
                raise ValueError("bore must be [6][nsamp]")
            if self.det_off.dim() != 2 or self.det_off.shape[0] != 4:
                raise ValueError("det_off must be [4][ndet]")
            self.ndet, self.nsamp = int(self.det_off.shape[1]), int(self.bore.shape[1])
        self.npix = self.ny * self.nx
        self.tod_dtype = {"f32": MM_F32, "bf16": MM_BF16, "f64": MM_F64}[tod_dtype]
        # dtype of the timestream handed to rhs (bf16: rounded to nearest even)
        self.real_dtype = {"f32": torch.float32, "bf16": torch.bfloat16,
                           "f64": torch.float64}[tod_dtype]
        d = mm_scan_desc()
        d.ncomp, d.ny, d.nx, d.ndet = self.ncomp, self.ny, self.nx, self.ndet
        d.tod_dtype = self.tod_dtype
        d.nsamp = self.nsamp
        d.fsample = float(getattr(inputs, "fsample", 0.0))
        d.pix = self.pix.data_ptr() if self.pix is not None else None
        if pointing == "boresight":
            d.pointing = MM_POINT_BORESIGHT
            d.bore = self.bore.data_ptr()
            d.det_off = self.det_off.data_ptr()
        d.cos2psi = self.cos2psi.data_ptr() if self.cos2psi is not None else None
        d.sin2psi = self.sin2psi.data_ptr() if self.sin2psi is not None else None
        d.inv_noise = self.inv_noise.data_ptr()
        d.det_group = int(det_group)
        d.fft_m1 = int(fft_m1)
        d.fft_cols = int(fft_cols)
        d.mask_rcond = float(mask_rcond)
        d.scatter = {"auto": MM_SCATTER_AUTO, "atomic": MM_SCATTER_ATOMIC,
                     "samples": MM_SCATTER_SAMPLES}[scatter]
        d.acc = {"f64": MM_ACC_F64, "f32x2": MM_ACC_F32X2}[acc]
        d.pointing_code = {"auto": MM_PTC_AUTO, "off": MM_PTC_OFF}[pointing_code]
        edges = getattr(inputs, "corr_edges", None)
        if edges is not None:   # inter-detector correlated inverse noise
            self.corr_edges = np.ascontiguousarray(edges, dtype=np.int32)   # host, copied at create
            self.corr_V = up(inputs.corr_V, torch.float32)
            d.corr_nbins = len(self.corr_edges) - 1
            d.corr_rank = int(self.corr_V.shape[-1])
            d.corr_edges = self.corr_edges.ctypes.data
            d.corr_V = self.corr_V.data_ptr()
        nbytes = mm_scan_workspace_bytes(d)
        if nbytes == 0:
            raise MMError(MM_EINVAL, "mm_scan_workspace_bytes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        d.workspace = (base + 255) // 256 * 256
        d.workspace_bytes = nbytes
        self.desc = d
        self.handle = mm_create_scan(d, stream)

    # convenience wrappers (allocate outputs, same names)
    def new_map(self):
        return torch.zeros(self.ncomp * self.npix, dtype=torch.float64, device=self.device)

    def apply_A(self, x, y=None, stream=None):
        y = self.new_map() if y is None else y
        mm_apply_A(self.handle, x, y, stream)
        return y

    def rhs(self, tod, b=None, stream=None):
        b = self.new_map() if b is None else b
        tod = tod.to(device=self.device, dtype=self.real_dtype).contiguous()
        mm_rhs(self.handle, tod, b, stream)
        return b

    def build_precon(self, name, ref=None, sigma=0.0, symmetrize=True, eig_floor_rel=0.0,
                     tile=0, probe_sets=0, stream=None):
        """tile: side of the tiles of the "tiled" preconditioner; its device
        workspace is allocated here and held by this object.  probe_sets: 0
        probes every tile alone, s >= 2 shares probes among tiles s apart."""
        o = mm_precon_opts()
        o.ref_y, o.ref_x = (-1, -1) if ref is None else (int(ref[0]), int(ref[1]))
        o.gauss_sigma_px = float(sigma) if sigma else 0.0
        o.symmetrize = 1 if symmetrize else 0
        o.eig_floor_rel = float(eig_floor_rel)
        if name == "tiled":
            nb = mm_tiled_workspace_bytes(self.handle, tile)
            if nb == 0:
                raise ValueError(f"invalid tile size {tile} for a {self.ny} x {self.nx} map")
            self._tiled_ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
            o.tile = int(tile)
            o.tiled_workspace = self._tiled_ws.data_ptr()
            o.tiled_workspace_bytes = nb
            o.probe_sets = int(probe_sets)
        mm_build_precon(self.handle, PRECON[name], o, stream)

    def apply_precon(self, name, r, z=None, stream=None):
        z = self.new_map() if z is None else z
        if name == "circulant":
            mm_apply_precon_circulant(self.handle, r, z, stream)
        elif name == "tiled":
            mm_apply_precon_tiled(self.handle, r, z, stream)
        elif name == "learned":
            mm_apply_precon_learned(self.handle, r, z, stream)
        else:
            mm_apply_precon_binned(self.handle, PRECON[name], r, z, stream)
        return z

    def pcg(self, name, b, x=None, tol=1e-6, maxiter=5000, check_every=1, x0=False,
            history=True, snapshots=None, snap_every=0, graph=False, flexible=False, refine=0,
            true_residual=False, stream=None):
        x = self.new_map() if x is None else x
        o = _pcg_opts(tol, maxiter, check_every, x0, graph, flexible, refine, true_residual)
        if snapshots is not None:
            o.snapshots = _ptr(snapshots, torch.float64, name="snapshots").value
            o.snap_every = int(snap_every)
            o.max_snaps = snapshots.numel() // (self.ncomp * self.npix)
        st, res = mm_pcg_solve(self.handle, PRECON[name], b, x, o, stream,
                               history_len=maxiter if history else 0)
        res["x"] = x
        return res

    def judge(self, candidates, b, x=None, tol=1e-6, maxiter=5000, check_every=1, graph=False,
              refine=0):
        """mm_precon_judge: one solve per candidate; returns (chosen name,
        {name: result dict}, x of the chosen solve)."""
        x = self.new_map() if x is None else x
        o = _pcg_opts(tol, maxiter, check_every, False, graph, False, refine, False)
        _, chosen, out = mm_precon_judge(self.handle, candidates, b, x, o)
        names = {v: k for k, v in PRECON.items() if k not in ("none",)}
        names[PRECON["none"]] = "none"
        return names[chosen], {c if isinstance(c, str) else names[c]: r
                               for c, r in zip(candidates, out)}, x

    def attach_learned(self, learned):
        """Attach a Learned correction (None detaches); the scan keeps it alive."""
        mm_learned_attach(self.handle, None if learned is None else learned.handle)
        self._learned = learned

    def spectra(self, x, pixel_arcmin=0.5, dell=100.0, nbins=200, stream=None):
        """Binned flat-sky TT (EE, BB) spectra of the map x and the mode counts."""
        return mm_map_spectra(self.handle, x, pixel_arcmin, dell, nbins, self.ncomp, stream)

    def info(self):
        return mm_get_info(self.handle)

    def mask(self, stream=None):
        m = torch.empty(self.npix, dtype=torch.int32, device=self.device)
        mm_get_mask(self.handle, m, stream)
        return m

    def close(self):
        if getattr(self, "handle", None) is not None:
            mm_destroy_scan(self.handle)
            self.handle = None


class Learned:
    """A learned correction with its device workspace (owned here)."""

    def __init__(self, ncomp, ny, nx, batch, w1, w2, device="cuda", stream=None):
        self.ncomp, self.ny, self.nx, self.batch = ncomp, ny, nx, batch
        nbytes = mm_learned_workspace_bytes(ncomp, ny, nx, batch)
        if nbytes == 0:
            raise MMError(MM_EINVAL, "mm_learned_workspace_bytes")
        self._raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self._raw.data_ptr()) % 256
        self.workspace = self._raw[off: off + nbytes]
        self.handle = mm_learned_create(ncomp, ny, nx, batch, self.workspace, w1, w2, stream)

    def weights(self):
        return mm_learned_get(self.handle, self.ncomp)

    def train(self, r_w, t, e2, epochs=20, batch=16, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
              seed=0, shuffle=True, drop_last=False, stream=None):
        o = mm_train_opts()
        o.epochs, o.batch, o.lr, o.beta1, o.beta2, o.eps = epochs, batch, lr, beta1, beta2, eps
        o.seed, o.shuffle, o.drop_last = seed, int(shuffle), int(drop_last)
        return mm_learned_train(self.handle, r_w, t, e2, e2.numel(), o, stream)

    def loss(self, r_w, t, e2, stream=None):
        return mm_learned_loss(self.handle, r_w, t, e2, e2.numel(), stream)

    def close(self):
        if getattr(self, "handle", None) is not None:
            mm_learned_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pcg_batch(scans, name, bs, xs=None, tol=1e-6, maxiter=5000, check_every=8, graph=True,
              refine=0, true_residual=False, stream=None):
    """Solve several scans together (mm_pcg_solve_batch); returns the result
    dicts, each with its solution under "x"."""
    xs = [sc.new_map() for sc in scans] if xs is None else xs
    o = _pcg_opts(tol, maxiter, check_every, False, graph, False, refine, true_residual)
    _, out = mm_pcg_solve_batch([sc.handle for sc in scans], PRECON[name], bs, xs, o, stream)
    for r, x in zip(out, xs):
        r["x"] = x
    return out

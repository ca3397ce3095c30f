"""Plan autotuner: picks the four-step FFT split (fft_m1), the columns per
pass-1/3 block (fft_cols) and the detector-group size (det_group) of a scan
shape by timing mm_apply_A for each candidate plan on the GPU.

    best = tune(inputs, tod_dtype="f32")      # {"fft_m1": .., "fft_cols": .., "det_group": ..}
    scan = Scan(inputs, tod_dtype="f32", **best)

Results are cached per shape (ncomp, ny, nx, ndet, nsamp, tod_dtype, acc) in
a JSON file (default ~/.cache/paper_1309_7473_amd/autotune.json).  One-kernel
plans (nsamp/2 <= 8192) have nothing to tune and return {}.
"""

import json
import math
import os

ONE_KERNEL_MAX_M = 8192   # packed length handled by one block (kE * kNT)


def default_cache_path():
    root = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(root, "paper_1309_7473_amd", "autotune.json")


def _shape(inputs):
    """(ndet, nsamp) from the stored pointing [ndet][nsamp], else from the
    boresight model (bore [6][nsamp], det_off [4][ndet])."""
    pix = getattr(inputs, "pix", None)
    if pix is not None:
        return int(pix.shape[0]), int(pix.shape[1])
    return int(inputs.det_off.shape[1]), int(inputs.bore.shape[1])


def shape_key(inputs, tod_dtype, acc):
    ndet, nsamp = _shape(inputs)
    return f"{int(inputs.ncomp)}x{int(inputs.ny)}x{int(inputs.nx)}:{ndet}x{nsamp}:{tod_dtype}:{acc}"


def candidates(nsamp, ndet, tod_dtype="f32"):
    """Candidate plans for a four-step shape: every split the library accepts
    with M1 from 2^max(2, logM-12) to 2^min(10, logM-5), 8 or 16 columns, and
    the automatic detector group (about 512 MiB of pass buffer), half of it
    or a quarter."""
    M = nsamp // 2
    if M <= ONE_KERNEL_MAX_M:
        return []
    logM = int(round(math.log2(M)))
    cxb = {"f32": 8, "bf16": 4, "f64": 16}[tod_dtype]
    g_auto = max(1, min(ndet, (512 << 20) // (M * cxb)))
    groups = sorted({g_auto, max(1, g_auto // 2), max(1, g_auto // 4)})
    out = []
    for l1 in range(max(2, logM - 12), min(10, logM - 5) + 1):
        for cols in (8, 16):
            for g in groups:
                out.append({"fft_m1": 1 << l1, "fft_cols": cols, "det_group": g})
    return out


def _time_apply(scan, reps):
    import torch
    x = torch.zeros(scan.ncomp * scan.npix, dtype=torch.float64, device=scan.device)
    x.normal_(generator=torch.Generator(device=scan.device).manual_seed(0))
    y = scan.new_map()
    for _ in range(2):
        scan.apply_A(x, y)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        scan.apply_A(x, y)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def tune(inputs, tod_dtype="f32", acc="f64", reps=5, cache_path=None, use_cache=True,
         timer=None, verbose=False):
    """Returns the fastest plan's Scan keyword arguments.  timer(plan) -> seconds
    replaces the GPU timing (used by the CPU tests of the cache logic)."""
    key = shape_key(inputs, tod_dtype, acc)
    path = cache_path or default_cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return dict(cache[key]["plan"])
    ndet, nsamp = _shape(inputs)
    cands = candidates(nsamp, ndet, tod_dtype)
    if not cands:
        return {}
    if timer is None:
        timer = _gpu_timer(inputs, tod_dtype, acc, reps)
    results = []
    for plan in cands:
        try:
            t = timer(plan)
        except Exception as e:  # a plan the library rejects for this shape
            if verbose:
                print(f"autotune {key} {plan}: rejected ({e})", flush=True)
            continue
        results.append((t, plan))
        if verbose:
            print(f"autotune {key} {plan}: {t * 1e3:.3f} ms", flush=True)
    if not results:
        return {}
    t_best, best = min(results, key=lambda r: r[0])
    if use_cache:
        cache[key] = {"plan": best, "apply_s": t_best,
                      "tried": [{"plan": p, "apply_s": t} for t, p in results]}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
    return dict(best)


def _gpu_timer(inputs, tod_dtype, acc, reps):
    """Times one candidate at a time; the inputs go to the device once."""
    import torch
    from . import Scan
    dev = torch.device("cuda")

    class OnDevice:
        pass

    d = OnDevice()
    for name in ("ncomp", "ny", "nx", "fsample"):
        setattr(d, name, getattr(inputs, name, 0.0))

    def up(a, dt):
        if a is None:
            return None
        if isinstance(a, torch.Tensor):
            return a.to(device=dev, dtype=dt).contiguous()
        import numpy as np
        return torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dt)

    d.pix = up(inputs.pix, torch.int32)
    d.cos2psi = up(inputs.cos2psi, torch.float32)
    d.sin2psi = up(inputs.sin2psi, torch.float32)
    d.inv_noise = up(inputs.inv_noise, torch.float32)

    def timer(plan):
        scan = Scan(d, tod_dtype=tod_dtype, acc=acc, **plan)
        try:
            return _time_apply(scan, reps)
        finally:
            scan.close()
            del scan
            torch.cuda.empty_cache()

    return timer

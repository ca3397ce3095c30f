// The extern "C" entry points declared in include/mm.h: argument validation
// (before anything is enqueued), handle lifetime and the thread-local error
// message.  The compute lives in filter.hip, binned.hip, circulant.hip and
// pcg.hip.
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include <vector>

#include "mm_internal.h"

namespace mm {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

mm_status fail(mm_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

mm_status hip_check(hipError_t e, const char* what) {
  g_err = std::string("HIP error ") + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ") in " + what;
  return MM_EDEVICE;
}

static constexpr uint64_t kMagic = 0x6d6d5f7363616e31ull;  // "mm_scan1"

struct Handle {
  uint64_t magic;
  ScanImpl impl;
};

static bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

static mm_status validate_shape(const mm_scan_desc* d) {
  if (!d) return fail(MM_EINVAL, "desc is NULL");
  if (d->ncomp != 1 && d->ncomp != 3) return fail(MM_EINVAL, "ncomp must be 1 or 3");
  if (!pow2(d->ny) || !pow2(d->nx) || d->ny < 4 || d->nx < 4 || d->ny > 4096 || d->nx > 4096)
    return fail(MM_EINVAL, "ny and nx must be powers of two in [4, 4096]");
  if (d->ndet < 1) return fail(MM_EINVAL, "ndet must be >= 1");
  if (d->nsamp < 16 || d->nsamp > (int64_t(1) << 22) || (d->nsamp & 1))
    return fail(MM_EINVAL, "nsamp must be even and in [16, 2^22]");
  if (d->tod_dtype != MM_F32 && d->tod_dtype != MM_BF16 && d->tod_dtype != MM_F64)
    return fail(MM_EINVAL, "tod_dtype must be MM_F32, MM_BF16 or MM_F64");
  if (d->det_group < 0) return fail(MM_EINVAL, "det_group must be >= 0");
  if (d->fft_m1 < 0 || (d->fft_m1 > 0 && !pow2(d->fft_m1)))
    return fail(MM_EINVAL, "fft_m1 must be 0 or a power of two");
  if (d->fft_cols < 0 || (d->fft_cols > 0 && !pow2(d->fft_cols)))
    return fail(MM_EINVAL, "fft_cols must be 0 or a power of two");
  if (d->scatter != MM_SCATTER_AUTO && d->scatter != MM_SCATTER_ATOMIC &&
      d->scatter != MM_SCATTER_SAMPLES)
    return fail(MM_EINVAL, "scatter must be MM_SCATTER_AUTO, MM_SCATTER_ATOMIC or MM_SCATTER_SAMPLES");
  if (d->acc != MM_ACC_F64 && d->acc != MM_ACC_F32X2)
    return fail(MM_EINVAL, "acc must be MM_ACC_F64 or MM_ACC_F32X2");
  if (d->pointing_code != MM_PTC_AUTO && d->pointing_code != MM_PTC_OFF)
    return fail(MM_EINVAL, "pointing_code must be MM_PTC_AUTO or MM_PTC_OFF");
  if (d->acc == MM_ACC_F32X2 && d->scatter == MM_SCATTER_ATOMIC)
    return fail(MM_EINVAL, "acc = MM_ACC_F32X2 needs scatter = MM_SCATTER_AUTO");
  if (d->pointing != MM_POINT_STORED && d->pointing != MM_POINT_BORESIGHT)
    return fail(MM_EINVAL, "pointing must be MM_POINT_STORED or MM_POINT_BORESIGHT");
  if (d->pointing == MM_POINT_BORESIGHT && d->scatter == MM_SCATTER_ATOMIC)
    return fail(MM_EINVAL, "MM_POINT_BORESIGHT needs scatter = MM_SCATTER_AUTO");
  if (d->corr_rank < 0 || d->corr_rank > 16) return fail(MM_EINVAL, "corr_rank must be in [0, 16]");
  if (d->corr_rank > 0) {
    if (d->corr_nbins < 1 || d->corr_nbins > 4096)
      return fail(MM_EINVAL, "corr_nbins must be in [1, 4096]");
    if (!d->corr_edges) return fail(MM_EINVAL, "corr_edges is required when corr_rank > 0");
    const int32_t* e = d->corr_edges;
    if (e[0] != 0 || int64_t(e[d->corr_nbins]) != d->nsamp / 2 + 1)
      return fail(MM_EINVAL, "corr_edges must run from 0 to nsamp/2 + 1");
    for (int b = 0; b < d->corr_nbins; ++b)
      if (e[b + 1] <= e[b]) return fail(MM_EINVAL, "corr_edges must increase strictly");
  }
  return MM_OK;
}

static ScanImpl* get(mm_scan h) {
  Handle* hh = reinterpret_cast<Handle*>(h);
  if (!hh || hh->magic != kMagic) return nullptr;
  return &hh->impl;
}

}  // namespace mm

using namespace mm;

extern "C" {

const char* mm_last_error(void) { return g_err.c_str(); }

size_t mm_scan_workspace_bytes(const mm_scan_desc* desc) {
  if (validate_shape(desc) != MM_OK) return 0;
  Plan pl;
  Layout L;
  if (plan_and_layout(desc, &pl, &L) != MM_OK) return 0;
  return L.total;
}

mm_status mm_create_scan(const mm_scan_desc* desc, void* stream, mm_scan* out) {
  if (!out) return fail(MM_EINVAL, "out is NULL");
  *out = nullptr;
  mm_status r = validate_shape(desc);
  if (r != MM_OK) return r;
  if (!desc->inv_noise) return fail(MM_EINVAL, "inv_noise is required");
  if (desc->pointing == MM_POINT_BORESIGHT) {
    if (desc->pix || desc->cos2psi || desc->sin2psi)
      return fail(MM_EINVAL, "MM_POINT_BORESIGHT: pix, cos2psi and sin2psi must be NULL");
    if (!desc->bore || !desc->det_off)
      return fail(MM_EINVAL, "MM_POINT_BORESIGHT: bore and det_off are required");
    if (reinterpret_cast<uintptr_t>(desc->bore) % 16 != 0)
      return fail(MM_EINVAL, "bore must be 16-byte aligned");
  } else {
    if (!desc->pix) return fail(MM_EINVAL, "pix is required");
    if ((desc->ncomp == 3) != (desc->cos2psi != nullptr && desc->sin2psi != nullptr))
      return fail(MM_EINVAL, "cos2psi/sin2psi must be given iff ncomp == 3");
    if (desc->ncomp == 1 && (desc->cos2psi || desc->sin2psi))
      return fail(MM_EINVAL, "cos2psi/sin2psi must be NULL when ncomp == 1");
    // the timestream kernels read four samples at a time
    if (reinterpret_cast<uintptr_t>(desc->pix) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(desc->cos2psi) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(desc->sin2psi) % 16 != 0)
      return fail(MM_EINVAL, "pix, cos2psi and sin2psi must be 16-byte aligned");
  }
  if (desc->corr_rank > 0 && !desc->corr_V) return fail(MM_EINVAL, "corr_V is required");
  Plan pl;
  Layout L;
  if ((r = plan_and_layout(desc, &pl, &L)) != MM_OK) return r;
  if (!desc->workspace) return fail(MM_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(desc->workspace) % 256 != 0)
    return fail(MM_EINVAL, "workspace must be 256-byte aligned");
  if (desc->workspace_bytes < L.total)
    return fail(MM_ENOMEM, "workspace_bytes smaller than mm_scan_workspace_bytes()");
  Handle* h = new (std::nothrow) Handle;
  if (!h) return fail(MM_ENOMEM, "host allocation failed");
  h->magic = kMagic;
  ScanImpl& s = h->impl;
  s.d = *desc;
  s.nc = desc->ncomp;
  s.ny = desc->ny;
  s.nx = desc->nx;
  s.ndet = desc->ndet;
  s.npix = desc->ny * desc->nx;
  s.n = desc->nsamp;
  s.plan = pl;
  s.lay = L;
  s.ws = static_cast<char*>(desc->workspace);
  hipStream_t st = static_cast<hipStream_t>(stream);
  // binned_setup validates the inputs, builds the pixel-major index (when
  // the plan has one) and the binned blocks
  if ((r = upload_tables(&s, st)) != MM_OK || (r = binned_setup(&s, st)) != MM_OK ||
      (r = bore_setup(&s, st)) != MM_OK || (r = permute_inverse_spectrum(&s, st)) != MM_OK) {
    h->magic = 0;
    delete h;
    return r;
  }
  *out = reinterpret_cast<mm_scan>(h);
  return MM_OK;
}

void mm_destroy_scan(mm_scan scan) {
  Handle* h = reinterpret_cast<Handle*>(scan);
  if (!h || h->magic != kMagic) return;
  h->magic = 0;
  profile_free(&h->impl);
  delete h;
}

mm_status mm_rhs(mm_scan scan, const void* tod, double* b, void* stream) {
  ScanImpl* s = get(scan);
  if (!s) return fail(MM_EINVAL, "invalid scan handle");
  if (!tod || !b) return fail(MM_EINVAL, "tod and b are required");
  if (reinterpret_cast<uintptr_t>(tod) % 16 != 0) return fail(MM_EINVAL, "tod must be 16-byte aligned");
  return filter_pipeline(s, 1, tod, nullptr, b, static_cast<hipStream_t>(stream));
}

mm_status mm_apply_A(mm_scan scan, const double* x, double* y, void* stream) {
  ScanImpl* s = get(scan);
  if (!s) return fail(MM_EINVAL, "invalid scan handle");
  if (!x || !y) return fail(MM_EINVAL, "x and y are required");
  const size_t bytes = size_t(s->nc) * s->npix * 8;
  const char* xa = reinterpret_cast<const char*>(x);
  const char* ya = reinterpret_cast<const char*>(y);
  if (xa < ya + bytes && ya < xa + bytes) return fail(MM_EINVAL, "x and y overlap");
  return filter_pipeline(s, 0, nullptr, x, y, static_cast<hipStream_t>(stream));
}

mm_status mm_build_precon(mm_scan scan, int32_t precon, const mm_precon_opts* opts, void* stream) {
  ScanImpl* s = get(scan);
  if (!s) return fail(MM_EINVAL, "invalid scan handle");
  switch (precon) {
    case MM_M_NONE:
    case MM_M_JACOBI:
    case MM_M_BINNED:
    case MM_M_LEARNED:
      return MM_OK;
    case MM_M_CIRCULANT: {
      if (opts) {
        if ((opts->ref_y >= 0) != (opts->ref_x >= 0) || opts->ref_y >= s->ny || opts->ref_x >= s->nx)
          return fail(MM_EINVAL, "ref_y/ref_x out of range");
      }
      const auto t0 = std::chrono::steady_clock::now();
      const mm_status rc = circulant_build(s, opts, static_cast<hipStream_t>(stream));
      s->t_build_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      return rc;
    }
    case MM_M_TILED: {
      s->tiled_built = false;   // a previous build's workspace may be gone
      if (!opts) return fail(MM_EINVAL, "MM_M_TILED needs opts (tile and workspace)");
      if (!tiled_size_ok(s, opts->tile))
        return fail(MM_EINVAL, "tile must be a power of two in [8, min(ny, nx)] with <= 65535 tiles");
      if (!opts->tiled_workspace || reinterpret_cast<uintptr_t>(opts->tiled_workspace) % 256 != 0)
        return fail(MM_EINVAL, "tiled_workspace must be a 256-byte aligned device pointer");
      if (opts->tiled_workspace_bytes < tiled_workspace_bytes(s, opts->tile))
        return fail(MM_ENOMEM, "tiled_workspace_bytes below mm_tiled_workspace_bytes");
      if (opts->probe_sets < 0 || opts->probe_sets == 1)
        return fail(MM_EINVAL, "probe_sets must be 0 (each tile alone) or >= 2");
      const auto t0 = std::chrono::steady_clock::now();
      const mm_status rc = tiled_build(s, opts, static_cast<hipStream_t>(stream));
      s->t_build_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      return rc;
    }
    default:
      return fail(MM_EINVAL, "unknown preconditioner");
  }
}

mm_status mm_apply_precon_binned(mm_scan scan, int32_t precon, const double* r, double* z,
                                 void* stream) {
  ScanImpl* s = get(scan);
  if (!s) return fail(MM_EINVAL, "invalid scan handle");
  if (!r || !z) return fail(MM_EINVAL, "r and z are required");
  if (precon != MM_M_BINNED && precon != MM_M_JACOBI)
    return fail(MM_EINVAL, "precon must be MM_M_BINNED or MM_M_JACOBI");
  return binned_apply(s, precon == MM_M_JACOBI, r, z, static_cast<hipStream_t>(stream));
}

mm_status mm_apply_precon_circulant(mm_scan scan, const double* r, double* z, void* stream) {
  ScanImpl* s = get(scan);
  if (!s) return fail(MM_EINVAL, "invalid scan handle");
  if (!r || !z) return fail(MM_EINVAL, "r and z are required");
  return circulant_apply(s, r, z, static_cast<hipStream_t>(stream));
}

size_t mm_tiled_workspace_bytes(mm_scan scan, int32_t tile) {
  ScanImpl* s = get(scan);
  return s ? tiled_workspace_bytes(s, tile) : 0;
}

mm_status mm_apply_precon_tiled(mm_scan scan, const double* r, double* z, void* stream) {
  ScanImpl* s = get(scan);
  if (!s) return fail(MM_EINVAL, "invalid scan handle");
  if (!r || !z) return fail(MM_EINVAL, "r and z are required");
  return tiled_apply(s, r, z, static_cast<hipStream_t>(stream));
}

static mm_status check_solve(ScanImpl* s, int32_t precon, const double* b, double* x,
                             const mm_pcg_opts* opts) {
  if (!s) return fail(MM_EINVAL, "invalid scan handle");
  if (!b || !x || !opts) return fail(MM_EINVAL, "b, x and opts are required");
  if (!(opts->tol >= 0.0) || opts->maxiter < 0) return fail(MM_EINVAL, "bad tol or maxiter");
  if (precon < MM_M_NONE || precon > MM_M_TILED) return fail(MM_EINVAL, "unknown preconditioner");
  if (precon == MM_M_TILED && !s->tiled_built)
    return fail(MM_ENOTBUILT, "tiled preconditioner not built");
  if ((precon == MM_M_CIRCULANT || precon == MM_M_LEARNED) && !s->circ_built)
    return fail(MM_ENOTBUILT, "circulant preconditioner not built");
  if (precon == MM_M_LEARNED && !s->learned)
    return fail(MM_ENOTBUILT, "no learned correction attached");
  if (opts->snapshots == nullptr && opts->snap_every > 0)
    return fail(MM_EINVAL, "snap_every > 0 needs a snapshots buffer");
  const size_t bytes = size_t(s->nc) * s->npix * 8;
  const char* ba = reinterpret_cast<const char*>(b);
  const char* xa = reinterpret_cast<const char*>(x);
  if (ba < xa + bytes && xa < ba + bytes) return fail(MM_EINVAL, "b and x overlap");
  return MM_OK;
}

mm_status mm_pcg_solve(mm_scan scan, int32_t precon, const double* b, double* x,
                       const mm_pcg_opts* opts, mm_pcg_result* res, void* stream) {
  ScanImpl* s = get(scan);
  const mm_status rc = check_solve(s, precon, b, x, opts);
  if (rc != MM_OK) return rc;
  return pcg_solve(s, precon, b, x, opts, res, static_cast<hipStream_t>(stream));
}

mm_status mm_precon_judge(mm_scan scan, const int32_t* candidates, int32_t n, const double* b,
                          double* x, const mm_pcg_opts* opts, mm_pcg_result* res, int32_t* chosen,
                          void* stream) {
  ScanImpl* s = get(scan);
  if (!candidates || n < 1 || n > 16 || !chosen)
    return fail(MM_EINVAL, "candidates (1..16) and chosen are required");
  if (opts && opts->snapshots) return fail(MM_EINVAL, "the judge takes no snapshots");
  for (int i = 0; i < n; ++i) {
    const mm_status rc = check_solve(s, candidates[i], b, x, opts);
    if (rc != MM_OK) return rc;
  }
  return precon_judge(s, candidates, n, b, x, opts, res, chosen, static_cast<hipStream_t>(stream));
}

mm_status mm_pcg_solve_batch(const mm_scan* scans, int32_t n, int32_t precon,
                             const double* const* b, double* const* x, const mm_pcg_opts* opts,
                             mm_pcg_result* res, int32_t* status, void* stream) {
  if (n < 1 || !scans || !b || !x || !opts) return fail(MM_EINVAL, "scans, b, x, opts and n >= 1 are required");
  std::vector<ScanImpl*> ss(n);
  for (int i = 0; i < n; ++i) {
    ss[i] = get(scans[i]);
    const mm_status rc = check_solve(ss[i], precon, b[i], x[i], opts);
    if (rc != MM_OK) return rc;
    for (int j = 0; j < i; ++j)
      if (ss[j] == ss[i]) return fail(MM_EINVAL, "a scan appears twice in the batch");
  }
  std::vector<mm_status> st(n, MM_OK);
  const mm_status rc = pcg_solve_batch(ss.data(), n, precon, b, x, opts, res, st.data(),
                                       static_cast<hipStream_t>(stream));
  if (status)
    for (int i = 0; i < n; ++i) status[i] = st[i];
  return rc;
}

mm_status mm_map_spectra(mm_scan scan, const double* x, double pixel_arcmin, double dell,
                         int32_t nbins, double* spectra, double* counts, void* stream) {
  ScanImpl* s = get(scan);
  if (!s) return fail(MM_EINVAL, "invalid scan handle");
  if (!x || !spectra) return fail(MM_EINVAL, "x and spectra are required");
  if (!(pixel_arcmin > 0.0) || !(dell > 0.0) || !std::isfinite(pixel_arcmin) || !std::isfinite(dell))
    return fail(MM_EINVAL, "pixel_arcmin and dell must be positive");
  if (nbins < 1 || nbins > kSpecMaxBins) return fail(MM_EINVAL, "nbins must be in [1, 512]");
  return map_spectra(s, x, pixel_arcmin, dell, nbins, spectra, counts,
                     static_cast<hipStream_t>(stream));
}

mm_status mm_map_spectra_noalloc(mm_scan scan, const double* x, double pixel_arcmin, double dell,
                                 int32_t nbins, double* spectra, double* counts, void* stream) {
  ScanImpl* s = get(scan);
  if (!s) return fail(MM_EINVAL, "invalid scan handle");
  if (!x || !spectra) return fail(MM_EINVAL, "x and spectra are required");
  if (!(pixel_arcmin > 0.0) || !(dell > 0.0) || !std::isfinite(pixel_arcmin) || !std::isfinite(dell))
    return fail(MM_EINVAL, "pixel_arcmin and dell must be positive");
  if (nbins < 1 || nbins > kSpecMaxBins) return fail(MM_EINVAL, "nbins must be in [1, 512]");
  return map_spectra_noalloc(s, x, pixel_arcmin, dell, nbins, spectra, counts,
                             static_cast<hipStream_t>(stream));
}

mm_status mm_anorm_error_estimate(const double* alpha, const double* rho, int32_t n, int32_t delay,
                                  double* est) {
  if (n < 0 || delay < 1) return fail(MM_EINVAL, "n must be >= 0 and delay >= 1");
  if (n >= delay && (!alpha || !rho || !est)) return fail(MM_EINVAL, "alpha, rho and est are required");
  for (int k = 0; k + delay <= n; ++k) {
    double e = 0.0;
    for (int j = k; j < k + delay; ++j) e += alpha[j] * rho[j];
    est[k] = e;
  }
  return MM_OK;
}

mm_status mm_spectrum_cv_error(const double* c_iter, const double* c_input, const double* counts,
                               int32_t ncomp, int32_t nbins, double* err) {
  if (ncomp < 1 || nbins < 1) return fail(MM_EINVAL, "ncomp and nbins must be >= 1");
  if (!c_iter || !c_input || !counts || !err)
    return fail(MM_EINVAL, "c_iter, c_input, counts and err are required");
  for (int c = 0; c < ncomp; ++c)
    for (int b = 0; b < nbins; ++b) {
      const int i = c * nbins + b;
      const double half = 0.5 * counts[b];
      if (half > 0.0 && c_input[i] > 0.0)
        err[i] = std::fabs(c_iter[i] - c_input[i]) / (c_input[i] * std::sqrt(2.0 / half));
      else
        err[i] = std::nan("");
    }
  return MM_OK;
}

mm_status mm_cv_crossing_step(const double* steps, const double* errors, int32_t n,
                              double threshold, int32_t block, double* step, int32_t* found) {
  if (n < 0 || block < 1) return fail(MM_EINVAL, "n must be >= 0 and block >= 1");
  if (!found || !step || (n > 0 && (!steps || !errors)))
    return fail(MM_EINVAL, "steps, errors, step and found are required");
  *found = 0;
  double prev_c = 0.0, prev_v = 0.0;
  for (int b0 = 0, j = 0; b0 < n; b0 += block, ++j) {
    const int b1 = b0 + block < n ? b0 + block : n;
    double cs = 0.0, vs = 0.0;
    for (int i = b0; i < b1; ++i) {
      cs += steps[i];
      vs += errors[i];
    }
    const double cen = cs / (b1 - b0), val = vs / (b1 - b0);
    if (val <= threshold) {
      if (j == 0) {
        *step = cen;
      } else {
        const double t = (prev_v - threshold) / (prev_v - val);
        *step = prev_c + t * (cen - prev_c);
      }
      *found = 1;
      return MM_OK;
    }
    prev_c = cen;
    prev_v = val;
  }
  return MM_OK;
}

mm_status mm_get_info(mm_scan scan, mm_scan_info* out) {
  ScanImpl* s = get(scan);
  if (!s || !out) return fail(MM_EINVAL, "invalid scan handle or out");
  out->n_active = s->n_active;
  out->ref_pixel = s->circ_built ? s->ref_pixel : -1;
  out->n_floored = s->n_floored;
  out->det_group = s->plan.G;
  out->fft_m1 = s->plan.single ? 1 : s->plan.M1;
  out->fft_m2 = s->plan.single ? (1 << s->plan.logM) : (1 << s->plan.logM2);
  out->fft_cols = s->plan.single ? 0 : (1 << s->plan.logC);
  out->single_pass = s->plan.single ? 1 : 0;
  out->csr = !s->plan.csr ? 0 : s->plan.rle ? 2 : 1;
  out->workspace_bytes = s->lay.total;
  out->gather_weights = (!s->plan.csr || s->nc != 3) ? -1 : !s->plan.csr_w ? 1 : s->csr_ang ? 2 : 0;
  out->pass1_pointing = s->plan.otf ? 1 : s->ptc_ready ? 3 : s->ang_t_ready ? 2 : 0;
  out->t_build_s = s->t_build_s;
  return MM_OK;
}

mm_status mm_get_mask(mm_scan scan, int32_t* dst, void* stream) {
  ScanImpl* s = get(scan);
  if (!s || !dst) return fail(MM_EINVAL, "invalid scan handle or dst");
  MM_HIP(hipMemcpyAsync(dst, s->ws + s->lay.mask, size_t(s->npix) * 4, hipMemcpyDeviceToDevice,
                        static_cast<hipStream_t>(stream)));
  return MM_OK;
}

size_t mm_learned_workspace_bytes(int32_t ncomp, int32_t ny, int32_t nx, int32_t batch) {
  if ((ncomp != 1 && ncomp != 3) || ny < 1 || nx < 1 || batch < 1) {
    fail(MM_EINVAL, "bad learned-correction shape");
    return 0;
  }
  return learned_workspace_bytes(ncomp, ny, nx, batch);
}

mm_status mm_learned_create(int32_t ncomp, int32_t ny, int32_t nx, int32_t batch, void* workspace,
                            size_t workspace_bytes, const float* w1, const float* w2, void* stream,
                            mm_learned* out) {
  if (!out) return fail(MM_EINVAL, "out is NULL");
  *out = nullptr;
  if ((ncomp != 1 && ncomp != 3) || ny < 1 || nx < 1 || batch < 1)
    return fail(MM_EINVAL, "bad learned-correction shape");
  if (!w1 || !w2 || !workspace) return fail(MM_EINVAL, "w1, w2 and workspace are required");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(MM_EINVAL, "workspace must be 256-byte aligned");
  if (workspace_bytes < learned_workspace_bytes(ncomp, ny, nx, batch))
    return fail(MM_ENOMEM, "workspace_bytes smaller than mm_learned_workspace_bytes()");
  return learned_create(ncomp, ny, nx, batch, workspace, workspace_bytes, w1, w2,
                        static_cast<hipStream_t>(stream), out);
}

void mm_learned_destroy(mm_learned learned) { learned_destroy(learned); }

mm_status mm_learned_get(mm_learned learned, float* w1, float* w2) {
  if (!w1 || !w2) return fail(MM_EINVAL, "w1 and w2 are required");
  return learned_get(learned, w1, w2);
}

mm_status mm_learned_attach(mm_scan scan, mm_learned learned) {
  ScanImpl* s = get(scan);
  if (!s) return fail(MM_EINVAL, "invalid scan handle");
  if (learned) {
    mm_status r = learned_check(learned, s->nc, s->ny, s->nx);
    if (r != MM_OK) return r;
  }
  s->learned = learned;
  return MM_OK;
}

mm_status mm_learned_make_pair(mm_scan scan, const double* x_f, const double* x_k, float* r_w,
                               float* t, float* e2, void* stream) {
  ScanImpl* s = get(scan);
  if (!s) return fail(MM_EINVAL, "invalid scan handle");
  if (!x_f || !x_k || !r_w || !t || !e2) return fail(MM_EINVAL, "null argument");
  return learned_make_pair(s, x_f, x_k, r_w, t, e2, static_cast<hipStream_t>(stream));
}

mm_status mm_learned_train(mm_learned learned, const float* r_w, const float* t, const float* e2,
                           int64_t npairs, const mm_train_opts* opts, double* loss_history,
                           void* stream) {
  if (!r_w || !t || !e2 || !opts) return fail(MM_EINVAL, "null argument");
  if (opts->epochs < 0 || !(opts->lr >= 0.0)) return fail(MM_EINVAL, "bad training options");
  return learned_train(learned, r_w, t, e2, npairs, opts, loss_history,
                       static_cast<hipStream_t>(stream));
}

mm_status mm_learned_loss(mm_learned learned, const float* r_w, const float* t, const float* e2,
                          int64_t npairs, double* loss, void* stream) {
  if (!r_w || !t || !e2 || !loss || npairs < 1) return fail(MM_EINVAL, "bad argument");
  return learned_loss(learned, r_w, t, e2, npairs, loss, static_cast<hipStream_t>(stream));
}

mm_status mm_learned_forward(mm_learned learned, const float* x, int32_t B, float* y, float* a1,
                             float* a2, float* a3, void* stream) {
  if (!x || !y) return fail(MM_EINVAL, "x and y are required");
  return learned_forward(learned, x, B, y, a1, a2, a3, static_cast<hipStream_t>(stream));
}

mm_status mm_learned_grad(mm_learned learned, const float* r_w, const float* t, const float* e2,
                          int32_t B, double* loss, float* g1, float* g2, void* stream) {
  if (!r_w || !t || !e2 || !loss || !g1 || !g2) return fail(MM_EINVAL, "null argument");
  return learned_grad(learned, r_w, t, e2, B, loss, g1, g2, static_cast<hipStream_t>(stream));
}

mm_status mm_apply_precon_learned(mm_scan scan, const double* r, double* z, void* stream) {
  ScanImpl* s = get(scan);
  if (!s) return fail(MM_EINVAL, "invalid scan handle");
  if (!r || !z) return fail(MM_EINVAL, "r and z are required");
  if (!s->circ_built) return fail(MM_ENOTBUILT, "circulant preconditioner not built");
  return learned_apply(s, r, z, static_cast<hipStream_t>(stream));
}

mm_status mm_profile_enable(mm_scan scan, int32_t enable) {
  ScanImpl* s = get(scan);
  if (!s) return fail(MM_EINVAL, "invalid scan handle");
  return profile_enable(s, enable != 0);
}

mm_status mm_profile_stages(mm_scan scan, uint32_t mask) {
  ScanImpl* s = get(scan);
  if (!s) return fail(MM_EINVAL, "invalid scan handle");
  return profile_stages(s, mask);
}

mm_status mm_profile_read(mm_scan scan, mm_profile* out) {
  ScanImpl* s = get(scan);
  if (!s || !out) return fail(MM_EINVAL, "invalid scan handle or out");
  return profile_read(s, out);
}

}  // extern "C"

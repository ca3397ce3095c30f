// Preconditioned conjugate gradients for A m = b (paper eq. 2) with every
// scalar kept on the device.
//
//   r0 = b - A x0, z0 = M r0, p0 = z0, rho0 = r0.z0
//   loop:  s = A p;  alpha = rho / p.s;  x += alpha p;  r -= alpha s;
//          stop when ||r|| <= tol ||b||;  z = M r;  rho' = r.z;
//          beta = rho' / rho;  p = z + beta p
//
// The flexible (Polak-Ribiere) variant takes beta = z.(r' - r) / rho =
// -alpha (s.z) / rho instead, which keeps consecutive directions
// A-conjugate when M is only nearly symmetric (the learned correction, whose
// convolutions round to bfloat16); s.z is the second sum of the r.z kernel.
// On request the loop is followed by the true residual b - A x (one more
// A-apply) and, while that misses the tolerance, by restarts from x (at most
// opts->refine of them): the recursive residual drifts from the true one by
// the rounding of the updates.
//
// Dot products are two-step reductions with a fixed summation order (block
// partials, then a 256-thread sum of the partials: for p.s and r.z
// redundantly in every block of the x/r and p updates that consume them, for
// ||r||^2 in block 0 of the next dot kernel, at the start in one-block
// kernels), so a solve is bit-reproducible.  Under
// MM_ACC_F32X2 (template CF) the products and sums are compensated float32
// pairs: each double is split into hi + lo floats, products take their fma
// error, sums are error-free, and a block partial is stored as (hi, lo) in
// the 8 bytes of its double slot.  The kernels read
// a `done` flag that the reductions set on convergence or breakdown
// (p.s <= 0, rho <= 0 or a non-finite scalar); after it, updates are no-ops,
// so the host only needs to look every check_every iterations.
#include <chrono>
#include <memory>
#include <vector>

#include "mm_device.h"
#include "mm_internal.h"

namespace mm {

constexpr int kRedBlocks = 512;

// block partial of NV sums, each as a double or as a float-float pair
template <bool CF>
struct Acc2 {
  double d[2] = {0.0, 0.0};
  F2 f[2] = {F2{0.f, 0.f}, F2{0.f, 0.f}};
  __device__ __forceinline__ void add_prod(int i, double x, double y) {
    if constexpr (CF)
      f2_fma_acc(f[i], f2_split(x), f2_split(y));
    else
      d[i] += x * y;
  }
  // block-reduce and store the block's two partials
  __device__ __forceinline__ void store(double* part) {
    __shared__ double sm[32];
    if constexpr (CF) {
      block_sum_f2<2>(f, reinterpret_cast<F2*>(sm));
      if (threadIdx.x == 0) {
        reinterpret_cast<F2*>(part)[2 * blockIdx.x] = f[0];
        reinterpret_cast<F2*>(part)[2 * blockIdx.x + 1] = f[1];
      }
    } else {
      block_sum<2>(d, sm);
      if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = d[0];
        part[2 * blockIdx.x + 1] = d[1];
      }
    }
  }
};

// partial sums of a.b (and c.d if c != nullptr)
template <bool CF>
__global__ void __launch_bounds__(256) k_dot_partial(const double* __restrict__ a,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ c,
                                                     const double* __restrict__ d, int64_t n,
                                                     double* __restrict__ part) {
  Acc2<CF> v;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    v.add_prod(0, a[i], b[i]);
    if (c) v.add_prod(1, c[i], d[i]);
  }
  v.store(part);
}

// final sum of the block partials (cf: they are float-float pairs)
__device__ __forceinline__ void sum_partials(const double* part, int nb, double (&v)[2], double* sm,
                                             int cf) {
  if (cf) {
    F2 f[2] = {F2{0.f, 0.f}, F2{0.f, 0.f}};
    const F2* pf = reinterpret_cast<const F2*>(part);
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
      f[0] = f2_add(f[0], pf[2 * i]);
      f[1] = f2_add(f[1], pf[2 * i + 1]);
    }
    block_sum_f2<2>(f, reinterpret_cast<F2*>(sm));
    v[0] = f2_value(f[0]);
    v[1] = f2_value(f[1]);
    return;
  }
  v[0] = v[1] = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    v[0] += part[2 * i];
    v[1] += part[2 * i + 1];
  }
  block_sum<2>(v, sm);
}

// init: bb = b.b and rr = r.r; converged already if ||r0|| <= tol ||b||
__global__ void k_fin_init(const double* __restrict__ part, int nb, PcgDev* st, double* hist) {
  __shared__ double sm[32];
  double v[2];
  sum_partials(part, nb, v, sm, st->cf);
  if (threadIdx.x == 0) {
    st->bb = v[0];
    st->rr = v[1];
    st->iters = 0;
    st->breakdown = 0;
    st->done = 0;
    if (!isfinite(v[0]) || !isfinite(v[1])) {
      st->done = 1;  // non-finite right-hand side or start
      st->breakdown = 1;
      hist[0] = v[1];
    } else if (!(v[0] > 0.0)) {
      st->done = 1;  // b = 0: x = 0 solves it
      hist[0] = 0.0;
    } else {
      hist[0] = sqrt(v[1] / v[0]);
      if (v[1] <= st->tol2 * v[0]) st->done = 1;
    }
  }
}

// ||b - A x||^2 of the true-residual check
__global__ void k_fin_true(const double* __restrict__ part, int nb, PcgDev* st) {
  __shared__ double sm[32];
  double v[2];
  sum_partials(part, nb, v, sm, st->cf);
  if (threadIdx.x == 0) st->true_rr = v[0];
}

// rho0 = r0.z0
__global__ void k_fin_rho0(const double* __restrict__ part, int nb, PcgDev* st) {
  __shared__ double sm[32];
  double v[2];
  sum_partials(part, nb, v, sm, st->cf);
  if (threadIdx.x == 0) st->rho = st->rz = v[0];
}

__global__ void k_mask_vec(double* __restrict__ x, const int32_t* __restrict__ mask, int npix,
                           int nc) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix || mask[p]) return;
  for (int a = 0; a < nc; ++a) x[int64_t(a) * npix + p] = 0.0;
}

// alpha = rho / p.s from the p.s partials (every block sums them in the same
// order, so all agree; block 0 records alpha, or the breakdown), then
// x += alpha p ; r -= alpha s ; partial r.r into part_rr (a buffer other
// than part_ps, which the other blocks may still be reading)
template <bool CF>
__global__ void __launch_bounds__(256) k_update_xr(double* __restrict__ x, double* __restrict__ r,
                                                   const double* __restrict__ p,
                                                   const double* __restrict__ s, int64_t n,
                                                   PcgDev* st, const double* part_ps, int nb,
                                                   double* __restrict__ part_rr) {
  if (st->done) return;   // uniform: set only by earlier kernels, or below when every block returns
  __shared__ double sm[32];
  __shared__ double ps_all;
  double ps2[2];
  sum_partials(part_ps, nb, ps2, sm, st->cf);   // the total is in thread 0
  if (threadIdx.x == 0) ps_all = ps2[0];
  __syncthreads();
  // rho of this iteration: the last r.z (set by the p update or the start)
  const double ps = ps_all, rho = st->rz;
  const bool bad = !(ps > 0.0) || !(rho > 0.0) || !isfinite(ps) || !isfinite(rho);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->ps = ps;
    st->rho = rho;   // read by the history and by the p update's beta
    if (bad) {
      st->breakdown = 1;
      st->done = 1;
      st->alpha = 0.0;
    } else {
      st->alpha = rho / ps;
    }
  }
  if (bad) return;
  const double alpha = rho / ps;
  Acc2<CF> v;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * s[i];
    r[i] = ri;
    v.add_prod(0, ri, ri);
  }
  v.store(part_rr);
}

// ||r||^2 from the x/r update's partials: the iteration count, the history
// and the convergence test.  Run by one block (all its threads).
__device__ __forceinline__ void fin_rr(const double* part, int nb, PcgDev* st, double* hist,
                                       int hist_cap) {
  if (st->done) return;   // read by every thread before thread 0 can change it
  __shared__ double sm[32];
  double v[2];
  sum_partials(part, nb, v, sm, st->cf);
  if (threadIdx.x == 0) {
    const double rr = v[0];
    st->rr = rr;
    const int it = st->iters + 1;
    st->iters = it;
    if (it <= hist_cap) {
      hist[it] = sqrt(rr / st->bb);
      hist[(hist_cap + 1) + it - 1] = st->alpha;
      hist[2 * (hist_cap + 1) + it - 1] = st->rho;
    }
    if (!isfinite(rr)) {
      st->breakdown = 1;
      st->done = 1;
    } else if (rr <= st->tol2 * st->bb) {
      st->done = 1;
    }
  }
}

// r.z partials of the p update, with block 0 first finishing ||r||^2 (the
// iteration's bookkeeping) from the x/r update's partials
template <bool CF>
__global__ void __launch_bounds__(256) k_dot_rz(const double* __restrict__ r,
                                                const double* __restrict__ z,
                                                const double* __restrict__ s, int64_t n,
                                                double* __restrict__ part, PcgDev* st,
                                                const double* part_rr, int nb, double* hist,
                                                int hist_cap) {
  if (blockIdx.x == 0) fin_rr(part_rr, nb, st, hist, hist_cap);
  Acc2<CF> v;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    v.add_prod(0, r[i], z[i]);
    if (s) v.add_prod(1, s[i], z[i]);   // flexible beta: s.z as the second sum
  }
  v.store(part);
}

// rho' = r.z from the r.z partials (every block sums them in the same order),
// beta = rho' / rho, p = z + beta p.  Block 0 records rho' in rz and beta; rho
// itself is left for the next x/r update to set, since the other blocks read
// it here.
__global__ void __launch_bounds__(256) k_update_p(double* __restrict__ p, const double* __restrict__ z,
                                                  int64_t n, PcgDev* st, const double* part_rz,
                                                  int nb) {
  if (st->done) return;   // uniform: set only by earlier kernels
  __shared__ double sm[32];
  __shared__ double rz_all, sz_all;
  double v[2];
  sum_partials(part_rz, nb, v, sm, st->cf);   // the totals are in thread 0
  if (threadIdx.x == 0) {
    rz_all = v[0];
    sz_all = v[1];
  }
  __syncthreads();
  const double rz = rz_all;
  const double beta = st->flex ? -st->alpha * sz_all / st->rho : rz / st->rho;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->rz = rz;
    st->beta = beta;
  }
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = z[i] + beta * p[i];
}

__global__ void k_axpby(double* __restrict__ out, const double* __restrict__ a, double ca,
                        const double* __restrict__ b, double cb, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    out[i] = ca * a[i] + (b ? cb * b[i] : 0.0);
}

static int red_blocks(int64_t n) {
  int64_t b = (n + 1023) / 1024;
  if (b < 1) b = 1;
  if (b > kRedBlocks) b = kRedBlocks;
  return int(b);
}

static mm_status apply_precon_inner(ScanImpl* s, int precon, const double* r, double* z,
                                    hipStream_t st);

mm_status apply_precon(ScanImpl* s, int precon, const double* r, double* z, hipStream_t st) {
  hipEvent_t tok;
  prof_begin(s, st, &tok, kProfPrecon);
  const mm_status rc = apply_precon_inner(s, precon, r, z, st);
  prof_end(s, st, tok, kProfPrecon, int64_t(s->nc) * s->npix);
  return rc;
}

static mm_status apply_precon_inner(ScanImpl* s, int precon, const double* r, double* z,
                                    hipStream_t st) {
  const int64_t N = int64_t(s->nc) * s->npix;
  switch (precon) {
    case MM_M_NONE: {
      hipLaunchKernelGGL(k_axpby, dim3(red_blocks(N)), dim3(256), 0, st, z, r, 1.0,
                         static_cast<const double*>(nullptr), 0.0, N);
      MM_HIP(hipGetLastError());
      return MM_OK;
    }
    case MM_M_JACOBI:
      return binned_apply(s, 1, r, z, st);
    case MM_M_BINNED:
      return binned_apply(s, 0, r, z, st);
    case MM_M_CIRCULANT:
      return circulant_apply(s, r, z, st);
    case MM_M_LEARNED:
      return learned_apply(s, r, z, st);
    case MM_M_TILED:
      return tiled_apply(s, r, z, st);
    default:
      return fail(MM_EINVAL, "unknown preconditioner");
  }
}

// ------------------------------------------------------------- host driver
// One solve in flight.  pcg_start enqueues r0, z0, p0 and rho0 and reads the
// state back; pcg_iterate enqueues one iteration (eager, or one launch of the
// captured graph); pcg_poll reads the device scalars; pcg_finish fills the
// result.  A batch interleaves several runs, each on its own stream.
struct PcgRun {
  ScanImpl* s = nullptr;
  int precon = 0;
  const double* b = nullptr;
  double* x = nullptr;
  mm_pcg_opts o{};
  mm_pcg_result* res = nullptr;
  hipStream_t st = nullptr;
  int it = 0;
  bool flex = false;
  bool finished = false;
  int offset = 0;        // iterations of the earlier segments (restarts)
  int restarts = 0;
  double true_rel = -1.0;
  double t_setup = 0.0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  PcgDev h{};
  std::chrono::steady_clock::time_point t0;
  ~PcgRun() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

// the launches of one iteration (no host synchronisation, no memset/memcpy:
// safe to capture)
static mm_status pcg_iteration_launches(ScanImpl* s, int precon, bool flex, double* x,
                                        hipStream_t st) {
  const Layout& L = s->lay;
  const int64_t N = int64_t(s->nc) * s->npix;
  double* vec = s->at<double>(L.vec);
  double *r = vec, *z = vec + N, *p = vec + 2 * N, *sv = vec + 3 * N;
  double* part = s->at<double>(L.partials);
  PcgDev* dev = s->at<PcgDev>(L.pcg);
  double* hist = s->at<double>(L.hist);
  const int nb = red_blocks(N);
  const dim3 gb(nb), bb(256);
  const bool cf = s->plan.acc32;
  const double* none = nullptr;
  auto dot = [&](const double* a, const double* b2) {
    if (cf)
      hipLaunchKernelGGL(k_dot_partial<true>, gb, bb, 0, st, a, b2, none, none, N, part);
    else
      hipLaunchKernelGGL(k_dot_partial<false>, gb, bb, 0, st, a, b2, none, none, N, part);
  };
  mm_status rc;
  // s = A p
  if ((rc = filter_pipeline(s, 0, nullptr, p, sv, st)) != MM_OK) return rc;
  dot(p, sv);
  // alpha is formed inside the update (no separate finalisation launch); its
  // r.r partials go to the second half of the partials region
  double* part_rr = part + 2 * kMaxPartials;
  if (cf)
    hipLaunchKernelGGL(k_update_xr<true>, gb, bb, 0, st, x, r, p, sv, N, dev, part, nb, part_rr);
  else
    hipLaunchKernelGGL(k_update_xr<false>, gb, bb, 0, st, x, r, p, sv, N, dev, part, nb, part_rr);
  if ((rc = apply_precon(s, precon, r, z, st)) != MM_OK) return rc;
  // r.z, with ||r||^2's bookkeeping in its block 0 (nothing between the x/r
  // update and here reads it)
  const double* sz = flex ? sv : nullptr;
  if (cf)
    hipLaunchKernelGGL(k_dot_rz<true>, gb, bb, 0, st, r, z, sz, N, part, dev, part_rr, nb, hist,
                       kHistCap);
  else
    hipLaunchKernelGGL(k_dot_rz<false>, gb, bb, 0, st, r, z, sz, N, part, dev, part_rr, nb, hist,
                       kHistCap);
  hipLaunchKernelGGL(k_update_p, gb, bb, 0, st, p, z, N, dev, part, nb);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

static mm_status pcg_poll(PcgRun& R) {
  MM_HIP(hipMemcpyAsync(&R.h, R.s->at<PcgDev>(R.s->lay.pcg), sizeof(PcgDev),
                        hipMemcpyDeviceToHost, R.st));
  MM_HIP(hipStreamSynchronize(R.st));
  return MM_OK;
}

static mm_status pcg_start(PcgRun& R) {
  if (R.offset == 0) R.t0 = std::chrono::steady_clock::now();
  ScanImpl* s = R.s;
  hipStream_t st = R.st;
  const Layout& L = s->lay;
  const int64_t N = int64_t(s->nc) * s->npix;
  double* vec = s->at<double>(L.vec);
  double *r = vec, *z = vec + N, *p = vec + 2 * N, *sv = vec + 3 * N;
  double* part = s->at<double>(L.partials);
  PcgDev* dev = s->at<PcgDev>(L.pcg);
  double* hist = s->at<double>(L.hist);
  const int nb = red_blocks(N);
  const dim3 gb(nb), bb(256);
  const double* none = nullptr;
  const bool cf = s->plan.acc32;
  auto dot = [&](const double* a, const double* b2, const double* c, const double* d) {
    if (cf)
      hipLaunchKernelGGL(k_dot_partial<true>, gb, bb, 0, st, a, b2, c, d, N, part);
    else
      hipLaunchKernelGGL(k_dot_partial<false>, gb, bb, 0, st, a, b2, c, d, N, part);
  };
  mm_status rc;
  PcgDev init{};
  init.tol2 = R.o.tol * R.o.tol;
  init.cf = cf ? 1 : 0;
  init.flex = R.flex ? 1 : 0;
  MM_HIP(hipMemcpyAsync(dev, &init, sizeof(PcgDev), hipMemcpyHostToDevice, st));
  // r = b - A x0  (or b), x0 = 0 unless use_x0
  if (R.o.use_x0) {
    hipLaunchKernelGGL(k_mask_vec, dim3((s->npix + 255) / 256), bb, 0, st, R.x,
                       s->at<int32_t>(L.mask), s->npix, s->nc);
    if ((rc = filter_pipeline(s, 0, nullptr, R.x, sv, st)) != MM_OK) return rc;
    hipLaunchKernelGGL(k_axpby, gb, bb, 0, st, r, R.b, 1.0, sv, -1.0, N);
  } else {
    hipLaunchKernelGGL(k_axpby, gb, bb, 0, st, r, R.b, 1.0, none, 0.0, N);
    hipLaunchKernelGGL(k_axpby, gb, bb, 0, st, R.x, R.b, 0.0, none, 0.0, N);
  }
  // inactive entries of b are ignored: r (and with it every later vector) is masked
  hipLaunchKernelGGL(k_mask_vec, dim3((s->npix + 255) / 256), bb, 0, st, r,
                     s->at<int32_t>(L.mask), s->npix, s->nc);
  MM_HIP(hipGetLastError());
  // ||b|| over the active entries (z is free until the first M r)
  hipLaunchKernelGGL(k_axpby, gb, bb, 0, st, z, R.b, 1.0, none, 0.0, N);
  hipLaunchKernelGGL(k_mask_vec, dim3((s->npix + 255) / 256), bb, 0, st, z,
                     s->at<int32_t>(L.mask), s->npix, s->nc);
  dot(z, z, r, r);
  hipLaunchKernelGGL(k_fin_init, dim3(1), bb, 0, st, part, nb, dev, hist);
  if ((rc = apply_precon(s, R.precon, r, z, st)) != MM_OK) return rc;
  hipLaunchKernelGGL(k_axpby, gb, bb, 0, st, p, z, 1.0, none, 0.0, N);
  dot(r, z, none, none);
  hipLaunchKernelGGL(k_fin_rho0, dim3(1), bb, 0, st, part, nb, dev);
  MM_HIP(hipGetLastError());
  if ((rc = pcg_poll(R)) != MM_OK) return rc;
  R.it = R.h.done ? R.o.maxiter : 0;
  if (R.o.graph && R.it < R.o.maxiter && !R.exec) {
    // capture one iteration; every later iteration is one graph launch
    s->capturing = true;
    MM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    rc = pcg_iteration_launches(s, R.precon, R.flex, R.x, st);
    const hipError_t ec = hipStreamEndCapture(st, &R.graph);
    s->capturing = false;
    if (rc != MM_OK) return rc;
    MM_HIP(ec);
    MM_HIP(hipGraphInstantiateWithFlags(&R.exec, R.graph, 0));
  }
  if (R.offset == 0)
    R.t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - R.t0).count();
  return MM_OK;
}

// enqueue one iteration (and the snapshot copy after it, if asked for)
static mm_status pcg_iterate(PcgRun& R) {
  if (R.exec) {
    MM_HIP(hipGraphLaunch(R.exec, R.st));
  } else {
    const mm_status rc = pcg_iteration_launches(R.s, R.precon, R.flex, R.x, R.st);
    if (rc != MM_OK) return rc;
  }
  ++R.it;
  const mm_pcg_opts& o = R.o;
  if (o.snapshots && o.snap_every > 0 && R.it % o.snap_every == 0 && R.it / o.snap_every <= o.max_snaps) {
    const int64_t N = int64_t(R.s->nc) * R.s->npix;
    MM_HIP(hipMemcpyAsync(o.snapshots + int64_t(R.it / o.snap_every - 1) * N, R.x, N * 8,
                          hipMemcpyDeviceToDevice, R.st));
  }
  return MM_OK;
}

// Reads the state of the segment that just ended and appends its history
// (entry 0 of a restarted segment, the true residual at the restart,
// replaces the last entry of the segment before).
static mm_status pcg_finish(PcgRun& R) {
  mm_status rc;
  if ((rc = pcg_poll(R)) != MM_OK) return rc;
  R.finished = true;
  const PcgDev& h = R.h;
  const int iters = h.iters;
  const int nh = iters < kHistCap ? iters : kHistCap;
  std::vector<double> hh(size_t(3) * (kHistCap + 1));
  MM_HIP(hipMemcpy(hh.data(), R.s->at<double>(R.s->lay.hist), hh.size() * 8, hipMemcpyDeviceToHost));
  const bool converged = h.done && !h.breakdown;
  if (R.res) {
    mm_pcg_result* res = R.res;
    const int off = R.offset;
    res->iters = off + iters;
    res->converged = converged ? 1 : 0;
    res->rel_resid = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
    if (iters == 0) res->rel_resid = h.bb > 0 ? hh[0] : 0.0;
    res->t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - R.t0).count();
    res->t_setup_s = R.t_setup;
    res->true_rel_resid = R.true_rel;
    res->restarts = R.restarts;
    if (res->history)
      for (int k = 0; k <= nh; ++k) res->history[off + k] = hh[k];
    if (res->alpha)
      for (int k = 0; k < nh; ++k) res->alpha[off + k] = hh[(kHistCap + 1) + k];
    if (res->rho)
      for (int k = 0; k < nh; ++k) res->rho[off + k] = hh[2 * (kHistCap + 1) + k];
  }
  if (h.breakdown) return fail(MM_EBREAKDOWN, "PCG breakdown (p.Ap <= 0, r.z <= 0 or non-finite)");
  if (!converged) {
    set_error("PCG did not reach the tolerance within maxiter");
    return MM_ENOCONV;
  }
  return MM_OK;
}

// ||b - A x|| / ||b|| over the active entries (one A-apply; z and s are free
// once the loop has stopped)
static mm_status pcg_true_residual(PcgRun& R, double* out) {
  ScanImpl* s = R.s;
  hipStream_t st = R.st;
  const Layout& L = s->lay;
  const int64_t N = int64_t(s->nc) * s->npix;
  double* vec = s->at<double>(L.vec);
  double *z = vec + N, *sv = vec + 3 * N;
  double* part = s->at<double>(L.partials);
  PcgDev* dev = s->at<PcgDev>(L.pcg);
  const int nb = red_blocks(N);
  const dim3 gb(nb), bb(256);
  const double* none = nullptr;
  mm_status rc;
  if ((rc = filter_pipeline(s, 0, nullptr, R.x, sv, st)) != MM_OK) return rc;
  hipLaunchKernelGGL(k_axpby, gb, bb, 0, st, z, R.b, 1.0, sv, -1.0, N);
  hipLaunchKernelGGL(k_mask_vec, dim3((s->npix + 255) / 256), bb, 0, st, z,
                     s->at<int32_t>(L.mask), s->npix, s->nc);
  if (s->plan.acc32)
    hipLaunchKernelGGL(k_dot_partial<true>, gb, bb, 0, st, z, z, none, none, N, part);
  else
    hipLaunchKernelGGL(k_dot_partial<false>, gb, bb, 0, st, z, z, none, none, N, part);
  hipLaunchKernelGGL(k_fin_true, dim3(1), bb, 0, st, part, nb, dev);
  MM_HIP(hipGetLastError());
  if ((rc = pcg_poll(R)) != MM_OK) return rc;
  *out = R.h.bb > 0 ? std::sqrt(R.h.true_rr / R.h.bb) : 0.0;
  return MM_OK;
}

static mm_status pcg_loop(PcgRun& R, int every) {
  mm_status rc;
  while (R.it < R.o.maxiter) {
    if ((rc = pcg_iterate(R)) != MM_OK) return rc;
    if (R.it % every == 0 || R.it == R.o.maxiter) {
      if ((rc = pcg_poll(R)) != MM_OK) return rc;
      if (R.h.done) break;
    }
  }
  return MM_OK;
}

// After a converged segment: the true residual (opts->true_residual or
// refine > 0) and, while it misses the tolerance, restarts from x with the
// iterations left, at most opts->refine times.  Returns the status of the
// last segment.
static mm_status pcg_check_and_refine(PcgRun& R, const mm_pcg_opts* o, mm_status rc) {
  const int every = o->check_every > 0 ? o->check_every : 1;
  while (rc == MM_OK && (o->true_residual || o->refine > 0)) {
    mm_status r2;
    if ((r2 = pcg_true_residual(R, &R.true_rel)) != MM_OK) return r2;
    if (R.res) R.res->true_rel_resid = R.true_rel;
    const int done_iters = R.offset + R.h.iters;
    if (R.true_rel <= o->tol || R.restarts >= o->refine || done_iters >= o->maxiter) break;
    // restart from x: r = b - A x, z = M r, p = z
    ++R.restarts;
    R.offset = done_iters;
    R.o.use_x0 = 1;
    R.o.maxiter = o->maxiter - done_iters;
    R.o.snapshots = nullptr;   // snapshots number the first segment's iterations only
    R.it = 0;
    R.finished = false;
    if ((r2 = pcg_start(R)) != MM_OK) return r2;
    if ((r2 = pcg_loop(R, every)) != MM_OK) return r2;
    rc = pcg_finish(R);
  }
  return rc;
}

// run on a private stream forked from / joined to the caller's (a captured
// stream must not be the null stream)
struct ForkedStream {
  hipStream_t caller, st = nullptr;
  hipEvent_t ev = nullptr;
  explicit ForkedStream(hipStream_t c) : caller(c) {}
  mm_status open() {
    MM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    MM_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    MM_HIP(hipEventRecord(ev, caller));
    MM_HIP(hipStreamWaitEvent(st, ev, 0));
    return MM_OK;
  }
  mm_status join() {
    MM_HIP(hipEventRecord(ev, st));
    MM_HIP(hipStreamWaitEvent(caller, ev, 0));
    return MM_OK;
  }
  ~ForkedStream() {
    if (st) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
    if (ev) (void)hipEventDestroy(ev);
  }
};

mm_status pcg_solve(ScanImpl* s, int precon, const double* b, double* x, const mm_pcg_opts* o,
                    mm_pcg_result* res, hipStream_t st) {
  ForkedStream fs(st);
  PcgRun R;
  R.s = s;
  R.precon = precon;
  R.b = b;
  R.x = x;
  R.o = *o;
  R.res = res;
  R.st = st;
  R.flex = precon == MM_M_LEARNED || o->flexible != 0;
  mm_status rc;
  if (o->graph) {
    if ((rc = fs.open()) != MM_OK) return rc;
    R.st = fs.st;
  }
  if ((rc = pcg_start(R)) != MM_OK) return rc;
  const int every = o->check_every > 0 ? o->check_every : 1;
  if ((rc = pcg_loop(R, every)) != MM_OK) return rc;
  rc = pcg_check_and_refine(R, o, pcg_finish(R));
  if (o->graph) {
    const mm_status rj = fs.join();
    if (rj != MM_OK) return rj;
  }
  return rc;
}

// The judge of preconditioners (and with it the fallback of a learned
// correction): one solve of A x = b per candidate, in the order given, each
// from x0 = 0 with the caller's options; the winner is the candidate that
// converged in the fewest iterations, the earlier one on ties (if none
// converged, the one with the smallest final residual).  Iteration counts are
// the paper's measure and, unlike wall times, repeatable.  The winner's
// solution is kept in the scan's spare map vector while the later candidates
// run and returned in x.
mm_status precon_judge(ScanImpl* s, const int32_t* cand, int n, const double* b, double* x,
                       const mm_pcg_opts* o, mm_pcg_result* res, int32_t* chosen, hipStream_t st) {
  const int64_t N = int64_t(s->nc) * s->npix;
  double* keep = s->at<double>(s->lay.vec) + 4 * N;   // spare vector: not used by PCG
  mm_pcg_opts oo = *o;
  oo.use_x0 = 0;
  int best = -1, best_iters = 0, best_conv = 0;
  double best_resid = 0.0;
  mm_status best_rc = MM_OK;
  for (int i = 0; i < n; ++i) {
    mm_pcg_result r{};
    if (res) r = res[i];   // the caller's history buffers, if any
    const mm_status rc = pcg_solve(s, cand[i], b, x, &oo, &r, st);
    if (rc < 0 && rc != MM_EBREAKDOWN) return rc;
    if (res) res[i] = r;
    const bool conv = rc == MM_OK && r.converged;
    const bool better = best < 0 || (conv && !best_conv) ||
                        (conv == bool(best_conv) &&
                         (conv ? r.iters < best_iters : r.rel_resid < best_resid));
    if (better) {
      best = i;
      best_iters = r.iters;
      best_conv = conv ? 1 : 0;
      best_resid = r.rel_resid;
      best_rc = rc;
      MM_HIP(hipMemcpyAsync(keep, x, size_t(N) * 8, hipMemcpyDeviceToDevice, st));
    }
  }
  MM_HIP(hipMemcpyAsync(x, keep, size_t(N) * 8, hipMemcpyDeviceToDevice, st));
  MM_HIP(hipStreamSynchronize(st));
  *chosen = cand[best];
  if (best_rc == MM_ENOCONV) set_error("no candidate reached the tolerance within maxiter");
  return best_rc;
}

// Independent solves interleaved: each run gets its own stream (forked from
// the caller's), every round enqueues check_every iterations of every
// unfinished run before any host read, so small scans overlap on the device.
mm_status pcg_solve_batch(ScanImpl* const* scans, int n, int precon, const double* const* b,
                          double* const* x, const mm_pcg_opts* o, mm_pcg_result* res,
                          mm_status* status, hipStream_t st) {
  std::vector<std::unique_ptr<ForkedStream>> fs;
  std::vector<PcgRun> R(n);
  mm_status rc;
  for (int i = 0; i < n; ++i) {
    fs.emplace_back(new ForkedStream(st));
    if ((rc = fs.back()->open()) != MM_OK) return rc;
    R[i].s = scans[i];
    R[i].precon = precon;
    R[i].b = b[i];
    R[i].x = x[i];
    R[i].o = *o;
    R[i].o.snapshots = nullptr;
    R[i].o.snap_every = 0;
    R[i].res = res ? &res[i] : nullptr;
    R[i].st = fs.back()->st;
    R[i].flex = precon == MM_M_LEARNED || o->flexible != 0;
  }
  for (int i = 0; i < n; ++i)
    if ((rc = pcg_start(R[i])) != MM_OK) return rc;
  const int every = o->check_every > 0 ? o->check_every : 1;
  for (;;) {
    bool any = false;
    for (int i = 0; i < n; ++i) {
      PcgRun& r = R[i];
      if (r.finished || r.h.done || r.it >= o->maxiter) continue;
      any = true;
      for (int k = 0; k < every && r.it < o->maxiter; ++k)
        if ((rc = pcg_iterate(r)) != MM_OK) return rc;
    }
    if (!any) break;
    for (int i = 0; i < n; ++i)
      if (!R[i].h.done && (rc = pcg_poll(R[i])) != MM_OK) return rc;
  }
  // first error of any run, else MM_ENOCONV if one did not converge
  mm_status worst = MM_OK;
  for (int i = 0; i < n; ++i) {
    const mm_status ri = pcg_check_and_refine(R[i], o, pcg_finish(R[i]));
    if (status) status[i] = ri;
    if (ri < 0 && worst >= 0) worst = ri;
    if (ri == MM_ENOCONV && worst == MM_OK) worst = MM_ENOCONV;
    if ((rc = fs[i]->join()) != MM_OK) return rc;
  }
  return worst;
}

}  // namespace mm

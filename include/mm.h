/*
 * mm.h - C ABI of the MI355X map-making library (libmm.so).
 *
 * The library solves the maximum-likelihood map-making equation
 *     (P^T N^-1 P) m = P^T N^-1 d                         (paper eq. 2)
 * for a pixelised I or I,Q,U sky map m, given detector timestreams d, a
 * nearest-pixel pointing matrix P with weights (1, cos 2psi, sin 2psi)
 * (eq. 1 and the Test setup section) and per-detector stationary noise N
 * (inverse power spectrum 1/N(f) per detector), by preconditioned conjugate
 * gradients with the binned (eq. 3-4), Jacobi (eq. 5) or circulant
 * "constant correlation" preconditioner (eq. 7-13).
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers (e.g. torch.Tensor.data_ptr() of a
 *     CUDA/HIP tensor) unless marked [host].
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it and the call returns without waiting unless the
 *     description says "synchronises".
 *   - Maps are float64 [ncomp][ny][nx], x fastest, pixel id p = y*nx + x.
 *     Only active pixels (hit at least once and, for I,Q,U, with a binned
 *     3x3 block of reciprocal condition number >= mask_rcond) are unknowns:
 *     every map the library writes is zero on inactive pixels, and inactive
 *     entries of input maps are ignored.
 *   - Timestream-shaped arrays are [ndet][nsamp], detector-major.
 *   - Errors: a status code is returned and no exception crosses the ABI.
 *     Arguments are validated before anything is enqueued, so an MM_EINVAL
 *     return has written nothing.  mm_last_error() gives a message for the
 *     last non-OK status on the calling thread.  Faults inside kernels
 *     surface as MM_EDEVICE at the next call that synchronises.
 *   - A handle is not thread-safe; distinct handles may be used concurrently
 *     on distinct streams.
 */
#ifndef MM_H
#define MM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mm_scan_s* mm_scan;   /* opaque, owned by the library */
typedef struct mm_learned_s* mm_learned;  /* opaque learned correction */

typedef enum {
  MM_OK = 0,
  MM_ENOCONV = 1,      /* non-fatal: PCG hit maxiter; x holds the last iterate */
  MM_EINVAL = -1,      /* bad argument; nothing was written */
  MM_ENOMEM = -2,      /* workspace too small */
  MM_EDEVICE = -3,     /* HIP runtime / kernel error */
  MM_ENOTBUILT = -4,   /* preconditioner requested before mm_build_precon */
  MM_EBREAKDOWN = -5   /* PCG breakdown (p.Ap <= 0, r.z <= 0 or non-finite);
                          x holds the last good iterate */
} mm_status;

typedef enum { MM_F32 = 0, MM_BF16 = 1, MM_F64 = 2 } mm_dtype;

/* Arithmetic of the long sums: the pixel accumulation of P^T and the PCG
 * inner products.  MM_ACC_F64: float64.  MM_ACC_F32X2: compensated float32
 * pairs (hi + lo, error-free sums and fma products, about 48 bits); the map
 * vectors stay float64 in memory. */
typedef enum { MM_ACC_F64 = 0, MM_ACC_F32X2 = 1 } mm_acc;

typedef enum {
  MM_M_NONE = 0,       /* identity */
  MM_M_JACOBI = 1,     /* eq. 5: per-pixel blocks of P^T P */
  MM_M_BINNED = 2,     /* eq. 3-4: per-pixel blocks of P^T diag(N^-1_tt) P */
  MM_M_CIRCULANT = 3,  /* eq. 8-13: Sigma^-1 F^-1 K(k)^-1 F Sigma^-T */
  MM_M_LEARNED = 4,    /* M_C + Sigma^-1 H^T H Sigma^-T (mm_learned_attach) */
  MM_M_TILED = 5       /* Summary section: overlapping tiles, each with its own
                          constant-correlation kernel, merged by a partition
                          of unity (mm_apply_precon_tiled) */
} mm_precon;

/* How a scan gives its pointing. */
typedef enum {
  MM_POINT_STORED = 0,     /* pix, cos2psi, sin2psi per sample */
  MM_POINT_BORESIGHT = 1   /* boresight track and detector offsets (Test setup
                              section); each sample's pixel and weights are
                              computed where they are needed */
} mm_pointing;

/* Description of one scan (one set of detector timestreams and pointing). */
typedef struct {
  int32_t ncomp;            /* 1 (I) or 3 (I,Q,U) */
  int32_t ny, nx;           /* map shape; powers of two in [4, 4096] */
  int32_t ndet;             /* detectors, >= 1 */
  int32_t tod_dtype;        /* mm_dtype of the timestream and its arithmetic:
                               MM_F32 (FFT and filter in float32),
                               MM_BF16 (d and the pass buffers between the
                               FFT kernels stored as bfloat16, rounded to
                               nearest even; FFT and filter math in float32),
                               MM_F64 (everything in float64) */
  int64_t nsamp;            /* samples per detector, 16 .. 2^22: a power of two, or
                               2^a 3^b 5^c (mixed-radix FFT: the one-kernel filter
                               up to nsamp/2 = 8192, beyond that a four-step with
                               rows 2^l and the factors 3 and 5 in columns of at
                               most 8192); correlated noise and boresight
                               pointing need a power of two */
  double  fsample;          /* sample rate in Hz (reporting only) */
  const int32_t* pix;       /* [ndet][nsamp] pixel id, -1 = off-map (zero row
                               of P); NULL with MM_POINT_BORESIGHT.  pix, cos2psi
                               and sin2psi are 16-byte aligned.  BORROWED:
                               must stay valid and unchanged until
                               mm_destroy_scan. */
  const float* cos2psi;     /* [ndet][nsamp] weight of Q; NULL iff ncomp == 1. BORROWED */
  const float* sin2psi;     /* [ndet][nsamp] weight of U; NULL iff ncomp == 1. BORROWED */
  const float* inv_noise;   /* [ndet][nsamp/2+1] 1/N_d(f_k) on the real-FFT
                               frequencies k = 0..nsamp/2; must be finite and
                               >= 0.  BORROWED */
  void*   workspace;        /* device memory of at least workspace_bytes, 256-byte
                               aligned; owned by the caller, used by the library
                               until mm_destroy_scan */
  size_t  workspace_bytes;
  int32_t det_group;        /* detectors per filter-pipeline group; 0 = automatic.
                               Bounds the timestream scratch in the workspace. */
  int32_t fft_m1;           /* four-step FFT split (0 = automatic): the packed
                               complex length nsamp/2 = fft_m1 * (nsamp/2/fft_m1);
                               ignored for mixed-radix nsamp */
  double  mask_rcond;       /* I,Q,U activity threshold on lambda_min/lambda_max of
                               the binned block; <= 0 selects 1e-3 */
  int32_t fft_cols;         /* columns per pass-1/3 block of the four-step FFT
                               (power of two, 0 = automatic) */
  int32_t scatter;          /* how P^T reaches the pixels in the multi-kernel
                               (four-step) pipeline: MM_SCATTER_AUTO = per-pixel
                               gather through a pixel-major index built at
                               creation (no atomics): with stored pointing and
                               groups of at most 2^28 samples the index holds runs
                               of consecutive samples (4 B per run, about 1 B a
                               sample on a raster scan; workspace sized for 4 B a
                               sample) and the gather reads the time-major weights
                               (plus 4 B/sample of workspace for their angle-coded
                               copy on the float32 and bfloat16 paths), otherwise
                               one 4 B entry a sample plus 8 B of weights;
                               MM_SCATTER_SAMPLES = the per-sample index always;
                               MM_SCATTER_ATOMIC = float64 atomic scatter (no
                               index).  The one-kernel path scatters atomically
                               unless acc = MM_ACC_F32X2. */
  int32_t acc;              /* mm_acc of the P^T accumulation and the PCG inner
                               products.  MM_ACC_F32X2 needs scatter =
                               MM_SCATTER_AUTO (it always takes the per-pixel
                               gather, also on the one-kernel path). */
  /* Inter-detector correlated inverse noise (the atmosphere and detector
   * correlations of the Test setup section's noise model).  corr_rank = 0:
   * detectors are independent and the three fields below are ignored.
   * corr_rank in 1..16: at real-FFT frequency k of bin b,
   *   N^-1(k) = diag(inv_noise[:, k]) - V_b V_b^T   (ndet x ndet),
   * which the caller keeps positive definite.  All detectors then form one
   * group (det_group is ignored) and the four-step pipeline runs with rows
   * of 512-2048 bins: nsamp in [2^13, 2^21]. */
  int32_t corr_rank;
  int32_t corr_nbins;       /* frequency bins, 1..4096 */
  const int32_t* corr_edges;/* [host] [corr_nbins + 1]: bin b holds edges[b] <= k <
                               edges[b+1]; edges[0] = 0, edges[corr_nbins] =
                               nsamp/2 + 1, strictly increasing.  Copied at create. */
  const float* corr_V;      /* [corr_nbins][ndet][corr_rank] device.  BORROWED */
  /* Pointing.  MM_POINT_STORED: pix (and cos2psi/sin2psi for I,Q,U) as above;
   * bore and det_off are ignored.  MM_POINT_BORESIGHT: pix, cos2psi and
   * sin2psi must be NULL and the library computes, in float64 without fused
   * multiply-add, for detector d at sample t (flat sky, pixel units, map
   * centre (c_y, c_x) = ((ny-1)/2, (nx-1)/2)):
   *   ry = (y_b - c_y) + dy_d,  rx = (x_b - c_x) + dx_d,
   *   py = (c_y + sin(phi) rx) + cos(phi) ry,  px = (c_x + cos(phi) rx) - sin(phi) ry,
   *   pixel (floor(py + 1/2), floor(px + 1/2)), off the map when outside,
   *   weights cos 2(psi_d + phi) = c2psi c2phi - s2psi s2phi and
   *           sin 2(psi_d + phi) = s2psi c2phi + c2psi s2phi.
   * The pixel-major index of P^T is then always used (scatter must not be
   * MM_SCATTER_ATOMIC): with MM_SCATTER_AUTO and groups of at most 2^28
   * samples the run-length index (4 B/sample of workspace at most) whose
   * gather computes the float64 weights from the model on the float64 path
   * and reads them as pixel-major 4-byte angles of the model's weights on
   * the float32 and bfloat16 paths (4 B/sample more); otherwise the
   * per-sample index (4 B/sample, plus 4 B/sample of angles on the float
   * paths). */
  int32_t pointing;         /* mm_pointing */
  const double* bore;       /* device [6][nsamp] float64, 16-byte aligned: y_b, x_b
                               (pixel coordinates), cos phi, sin phi, cos 2phi,
                               sin 2phi of the scan-angle turn.  BORROWED */
  const double* det_off;    /* device [4][ndet] float64: dy, dx (offsets from the
                               boresight before the turn), cos 2psi, sin 2psi.
                               BORROWED */
  int32_t pointing_code;    /* pass 1's copy of stored I,Q,U pointing whose weights
                               are angles (float32 and bfloat16 four-step paths,
                               nsamp a multiple of 64): MM_PTC_AUTO = chunk-coded
                               when every 64-sample chunk of every detector fits
                               (on-map pixels within 65534 of the chunk's smallest;
                               weight angles, as 2 psi 2^32 / 2 pi, less than 2^15
                               off the line through the chunk's first and last
                               on-map samples), 4 B a sample plus 16 B a chunk of
                               workspace, decoded to exactly the stored pixel and
                               angle; otherwise, and with MM_PTC_OFF, pass 1 reads
                               the stored pixels and the time-major angles (8 B a
                               sample) */
} mm_scan_desc;

enum { MM_PTC_AUTO = 0, MM_PTC_OFF = 1 };

enum { MM_SCATTER_AUTO = 0, MM_SCATTER_ATOMIC = 1, MM_SCATTER_SAMPLES = 2 };

/* Bytes of device workspace the scan needs (the caller allocates it and puts
 * the pointer in desc->workspace).  Only the shape fields and the tuning
 * fields (det_group, fft_m1, fft_cols, scatter, pointing, pointing_code,
 * tod_dtype, acc) are read.  Returns 0 and sets
 * mm_last_error() on an invalid description. */
size_t mm_scan_workspace_bytes(const mm_scan_desc* desc /*[host]*/);

/* Creates a scan handle: validates desc, uploads FFT twiddle tables into the
 * workspace, and computes on `stream` the per-detector binned weights
 * w_d = (N^-1)_tt (eq. 3-4), the hit counts, the binned and Jacobi blocks and
 * the active-pixel mask.  Synchronises `stream`.  *out receives the handle. */
mm_status mm_create_scan(const mm_scan_desc* desc /*[host]*/, void* stream,
                         mm_scan* out /*[host]*/);

/* Releases the handle (never frees caller memory).  NULL is a no-op. */
void mm_destroy_scan(mm_scan scan);

/* b = P^T N^-1 d (right-hand side of eq. 2) on the active pixels.
 * tod: [ndet][nsamp] in the scan's tod_dtype (float, bfloat16 bit patterns
 * as uint16, or double), 16-byte aligned.
 * b: [ncomp][ny][nx] float64, overwritten. */
mm_status mm_rhs(mm_scan scan, const void* tod, double* b, void* stream);

/* y = A x = P^T N^-1 P x (eq. 2), the per-iteration operator: a nearest-pixel
 * gather of x into timestreams, a per-detector real FFT, multiplication by
 * 1/N(f), the inverse FFT, and P^T back to pixels (per-pixel gather or
 * atomic scatter, see desc->scatter; accumulated in float64).
 * x, y: [ncomp][ny][nx] float64; y is overwritten; x and y must not overlap. */
mm_status mm_apply_A(mm_scan scan, const double* x, double* y, void* stream);

/* Options of the circulant preconditioner (Implementation, Regularization and
 * Polarization sections). */
typedef struct {
  int32_t ref_y, ref_x;     /* reference pixel; -1: the active pixel nearest
                               (ny/2, nx/2), smallest id on ties */
  double  gauss_sigma_px;   /* Gaussian taper of q (Regularization section);
                               <= 0 disables it */
  int32_t symmetrize;       /* 1: q(d) <- (q(d) + q(-d)^T)/2 and a Hermitian
                               eigenvalue floor; 0: eq. 12 literally (general
                               3x3 inverse per wavenumber, no floor) */
  double  eig_floor_rel;    /* floor = eig_floor_rel * max eigenvalue over all
                               wavenumbers (of the tile, for MM_M_TILED);
                               <= 0 selects 1e-6 */
  /* MM_M_TILED only (ref_y/ref_x and symmetrize are ignored there: each tile
   * probes the active pixel nearest its centre and is always symmetrised) */
  int32_t tile;             /* tile side T: a power of two, 8 <= T <= min(ny, nx);
                               tiles start every T/2 pixels.  Keep the taper
                               below about T/4: q is cut off at the tile's half
                               width, and a wider taper leaves K_t ill-conditioned */
  void*   tiled_workspace;  /* device memory of mm_tiled_workspace_bytes(scan,
                               tile) bytes, 256-byte aligned, owned by the caller
                               and kept alive (unchanged) while the preconditioner
                               is used */
  size_t  tiled_workspace_bytes;
  int32_t probe_sets;       /* 0: each tile's reference pixel is probed on its own
                               (ncomp A-applies per tile: the definition).
                               s >= 2: tiles whose tile row and column agree
                               modulo s share one A-apply per component (s^2
                               probe sets, same-set references >= s T/2 pixels
                               apart); cheaper, but each q_t then also holds the
                               other references' responses at its displacements,
                               damped only by distance and the taper.  1 is
                               rejected. */
} mm_precon_opts;

/* Builds a preconditioner on `stream`.  JACOBI, BINNED: per-pixel inverse
 * blocks (already prepared by mm_create_scan; this is a no-op).  CIRCULANT:
 * Sigma = B^(1/2) from the binned blocks (eq. 7), ncomp probes A e_(r,g)
 * (eq. 6), q (eq. 10/13), taper, optional symmetrisation, 2-D FFT (eq. 11),
 * per-wavenumber inverse.  Synchronises `stream`.  opts may be NULL for
 * defaults (no taper, symmetrize = 1, eig_floor_rel = 1e-6). */
mm_status mm_build_precon(mm_scan scan, int32_t precon /*mm_precon*/,
                          const mm_precon_opts* opts /*[host]*/, void* stream);

/* z = M r for the binned (eq. 3-4) or, with precon = MM_M_JACOBI, the Jacobi
 * (eq. 5) preconditioner: z_p = B_p^-1 r_p per active pixel. */
mm_status mm_apply_precon_binned(mm_scan scan, int32_t precon, const double* r,
                                 double* z, void* stream);

/* z = M_C r = Sigma^-1 F^-1 K^-1 F Sigma^-T r (eq. 12).  MM_ENOTBUILT if the
 * circulant preconditioner was not built. */
mm_status mm_apply_precon_circulant(mm_scan scan, const double* r, double* z,
                                    void* stream);

/* Bytes of device workspace the tiled preconditioner (Summary section) needs
 * for tile side `tile` on this scan's map: the per-tile inverse kernels
 * (ntiles T^2 ncomp^2 complex float64), the tile planes, one probe response
 * and small tables, with ntiles = (2 ny/T - 1)(2 nx/T - 1).  0 if the tile
 * size is invalid (not a power of two in [8, min(ny, nx)], or more than 65535
 * tiles). */
size_t mm_tiled_workspace_bytes(mm_scan scan, int32_t tile);

/* z = M_T r = Sigma^-1 [sum_t sqrt(W_t) F_t^-1 K_t^-1 F_t sqrt(W_t)] Sigma^-T r
 * (Summary section): per T x T tile t at stride T/2, the tile's own kernel
 * K_t (built like eq. 10-11 from a probe at the tile's reference pixel on the
 * tile's periodic displacement grid), merged by sin^2 weights W_t that sum to
 * one at every pixel.  r, z: [ncomp][ny][nx] float64.  MM_ENOTBUILT if
 * mm_build_precon(MM_M_TILED) has not run. */
mm_status mm_apply_precon_tiled(mm_scan scan, const double* r, double* z, void* stream);

typedef struct {
  double  tol;              /* stop when ||r||_2 <= tol ||b||_2 (recursive residual) */
  int32_t maxiter;          /* maximum A-applies in the loop */
  int32_t check_every;      /* read the residual on the host every k iterations (>= 1) */
  int32_t use_x0;           /* 1: start from the x passed in; 0: x0 = 0 */
  int32_t snap_every;       /* > 0: copy the iterate x_k into snapshots[k/snap_every - 1] */
  int32_t max_snaps;        /*      for k = snap_every, 2 snap_every, ... up to max_snaps */
  double* snapshots;        /* device [max_snaps][ncomp][ny][nx] float64, or NULL */
  int32_t graph;            /* 1: capture one iteration (A-apply, M, reductions and
                               updates) into a HIP graph on a private stream
                               forked from the caller's, and replay it; results
                               are those of the eager loop */
  int32_t flexible;         /* 1: beta = z_{k+1}.(r_{k+1} - r_k) / r_k.z_k (flexible,
                               Polak-Ribiere form; keeps consecutive directions
                               A-conjugate for a nearly symmetric M); always used
                               with MM_M_LEARNED.  0: beta = r_{k+1}.z_{k+1} / r_k.z_k */
  int32_t refine;           /* >= 0: after convergence of the recursive residual,
                               compute b - A x (one more A-apply) and, while
                               ||b - A x|| > tol ||b||, restart PCG from x with the
                               iterations left, at most `refine` times */
  int32_t true_residual;    /* 1: report ||b - A x|| / ||b|| (one more A-apply)
                               even with refine = 0 */
} mm_pcg_opts;

typedef struct {
  int32_t iters;            /* A-applies performed in the loop */
  int32_t converged;        /* 1 if ||r|| <= tol ||b|| was reached */
  double  rel_resid;        /* final recursive ||r|| / ||b|| */
  double  t_solve_s;        /* wall time of the solve */
  double* history;          /* [host] optional (may be NULL): ||r_k||/||b|| for
                               k = 0..iters, array of at least maxiter+1 */
  double* alpha;            /* [host] optional: alpha_k, k = 0..iters-1 */
  double* rho;              /* [host] optional: r_k.z_k, k = 0..iters-1 */
  double  t_setup_s;        /* wall time of the solve's set-up (r0, z0, p0, rho0 and
                               the graph capture), included in t_solve_s; the
                               preconditioner's own build time is
                               mm_scan_info.t_build_s */
  double  true_rel_resid;   /* ||b - A x|| / ||b|| of the returned x if computed
                               (refine > 0 or true_residual), else -1 */
  int32_t restarts;         /* restarts taken by `refine`; iters counts the
                               A-applies of every segment, history[k] at a restart
                               holds the true residual it started from */
} mm_pcg_result;

/* Solves A x = b by PCG (Introduction; textbook PCG with device-resident
 * scalars).  precon: MM_M_NONE, JACOBI, BINNED, CIRCULANT (built), LEARNED
 * (circulant built and a learned correction attached) or TILED (built).  b, x: [ncomp][ny][nx] float64 device arrays; x is overwritten
 * with the solution.  Synchronises `stream`.  Returns MM_OK, MM_ENOCONV or
 * MM_EBREAKDOWN (with res filled in all three cases). */
mm_status mm_pcg_solve(mm_scan scan, int32_t precon, const double* b, double* x,
                       const mm_pcg_opts* opts /*[host]*/,
                       mm_pcg_result* res /*[host]*/, void* stream);

/* The judge, and with it the fallback, of a learned correction (and of any
 * preconditioner choice): solves A x = b once with each candidate in
 * candidates[0..n-1] (1 <= n <= 16, each a preconditioner mm_pcg_solve
 * accepts on this scan, typically {MM_M_LEARNED, MM_M_CIRCULANT,
 * MM_M_BINNED}), each from x0 = 0 with *opts (no snapshots), and sets *chosen
 * to the candidate that reached opts->tol in the fewest iterations (the earlier
 * in the list on ties; if none converged, the smallest final residual).  Run it
 * on held-out data: the winner is the preconditioner to use for scans like it.
 * res: [host] n results (may be NULL; history arrays in them are filled).
 * x receives the winner's solution.  Synchronises.  Returns the winner's
 * status (MM_OK, MM_ENOCONV or MM_EBREAKDOWN) or an error. */
mm_status mm_precon_judge(mm_scan scan, const int32_t* candidates /*[host]*/, int32_t n,
                          const double* b, double* x, const mm_pcg_opts* opts /*[host]*/,
                          mm_pcg_result* res /*[host]*/, int32_t* chosen /*[host]*/, void* stream);

/* Independent solves of n scans, e.g. a batch of scans of uneven detector
 * count, length and map size.  Each run gets its own stream, forked from
 * `stream` and joined back; every round enqueues opts->check_every
 * iterations of every unfinished run before the host reads any state, so
 * the scans overlap on the device.  With opts->graph each run replays its
 * captured iteration.  No snapshots are taken.  scans: [host] n distinct
 * handles; b, x: [host] arrays of n device pointers ([ncomp][ny][nx] float64
 * of the matching scan); res: [host] n results; status: [host] n statuses or
 * NULL.  Synchronises.  Returns the first error of any run, else MM_ENOCONV
 * if a run stopped at maxiter, else MM_OK. */
mm_status mm_pcg_solve_batch(const mm_scan* scans /*[host]*/, int32_t n, int32_t precon,
                             const double* const* b /*[host]*/, double* const* x /*[host]*/,
                             const mm_pcg_opts* opts /*[host]*/, mm_pcg_result* res /*[host]*/,
                             int32_t* status /*[host]*/, void* stream);

/* ---- Learned correction to the circulant preconditioner (not in the paper):
 * M_L r = M_C r + Sigma^-1 H^T H Sigma^-T r, H = C2 o C1 with C1 (ncomp -> 16
 * channels) and C2 (16 -> 16) 5x5 same-padded correlations without bias,
 * H^T their exact adjoints (weights tied, so M_L is symmetric and M_L - M_C
 * positive semi-definite).  Convolutions run on bf16 MFMA with float32
 * accumulation; the float32 master weights are trained with Adam on
 * whitened pairs (r_w, t, ||e_w||^2) built by mm_learned_make_pair, loss
 * mean ||H^T H r_w - t||^2 / ||e_w||^2.  Weights: w1 [16][ncomp][5][5],
 * w2 [16][16][5][5] float32, row-major.  Images are [ncomp][ny][nx] float32. */
typedef struct {
  int32_t  epochs, batch;   /* batch <= the batch given to mm_learned_create */
  double   lr, beta1, beta2, eps;
  uint64_t seed;            /* pair shuffling */
  int32_t  shuffle, drop_last;
} mm_train_opts;

/* Device workspace for a learned correction on ny x nx maps with training
 * batches of up to `batch` pairs (activations, gradients, Adam state). */
size_t mm_learned_workspace_bytes(int32_t ncomp, int32_t ny, int32_t nx, int32_t batch);
mm_status mm_learned_create(int32_t ncomp, int32_t ny, int32_t nx, int32_t batch, void* workspace,
                            size_t workspace_bytes, const float* w1 /*[host]*/,
                            const float* w2 /*[host]*/, void* stream, mm_learned* out /*[host]*/);
void mm_learned_destroy(mm_learned learned);
mm_status mm_learned_get(mm_learned learned, float* w1 /*[host]*/, float* w2 /*[host]*/);
/* Attaches (or with NULL detaches) a learned correction of the scan's map
 * shape; MM_M_LEARNED then needs the circulant preconditioner built. */
mm_status mm_learned_attach(mm_scan scan, mm_learned learned);
/* One training pair from a converged x_f and an iterate x_k (device float64
 * maps): e = x_f - x_k, r = A e, r_w = Sigma^-T r, t = Sigma e - Sigma M_C r,
 * e2 = ||Sigma e||^2 (one float).  Needs the circulant preconditioner. */
mm_status mm_learned_make_pair(mm_scan scan, const double* x_f, const double* x_k, float* r_w,
                               float* t, float* e2, void* stream);
/* Adam epochs over npairs device pairs; loss_history [host, epochs] optional.
 * Synchronises. */
mm_status mm_learned_train(mm_learned learned, const float* r_w, const float* t, const float* e2,
                           int64_t npairs, const mm_train_opts* opts /*[host]*/,
                           double* loss_history /*[host]*/, void* stream);
/* Mean loss over npairs pairs (no update).  Synchronises. */
mm_status mm_learned_loss(mm_learned learned, const float* r_w, const float* t, const float* e2,
                          int64_t npairs, double* loss /*[host]*/, void* stream);
/* H^T H of B images x (device) into y, and optionally the intermediate
 * activations a1 = C1 x, a2 = C2 a1, a3 = C2^T a2 ([B][16][ny][nx]). */
mm_status mm_learned_forward(mm_learned learned, const float* x, int32_t B, float* y, float* a1,
                             float* a2, float* a3, void* stream);
/* Loss and weight gradients of B pairs without updating the weights;
 * g1, g2 [host] in the weight layouts.  Synchronises. */
mm_status mm_learned_grad(mm_learned learned, const float* r_w, const float* t, const float* e2,
                          int32_t B, double* loss /*[host]*/, float* g1 /*[host]*/,
                          float* g2 /*[host]*/, void* stream);
/* z = M_L r (circulant built, learned correction attached). */
mm_status mm_apply_precon_learned(mm_scan scan, const double* r, double* z, void* stream);

/* Flat-sky binned auto-spectra of a map, the power-spectrum diagnostic of the
 * Results section.  x: [ncomp][ny][nx] float64 device map; inactive pixels
 * count as zero (no apodisation).  Each component's unnormalised 2-D DFT X(k);
 * for I,Q,U also E = Q cos 2phi + U sin 2phi and B = -Q sin 2phi + U cos 2phi
 * with phi the wavevector angle.  Bin b holds the modes with
 * ell = 2 pi |k| / pixel_size in [b dell, (b+1) dell), |k| in cycles per
 * pixel, pixel_size = pixel_arcmin arcminutes; its value is
 * (pixel solid angle / ny nx) times the mean |X(k)|^2 over those modes.
 * spectra: [host] [ncomp == 3 ? 3 : 1][nbins] (TT, EE, BB); counts: [host]
 * [nbins] modes per bin (full Fourier plane), or NULL.  1 <= nbins <= 512.
 * Uses the preconditioner's FFT scratch (not concurrently with an apply on the
 * same handle).  Synchronises `stream`. */
mm_status mm_map_spectra(mm_scan scan, const double* x, double pixel_arcmin, double dell,
                         int32_t nbins, double* spectra /*[host]*/, double* counts /*[host]*/,
                         void* stream);

/* mm_map_spectra without any device memory from the caller or the scan's
 * workspace for its scratch: for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, results and synchronisation as mm_map_spectra; the Fourier
 * planes and bin partials live instead in one static device array of 64 MiB
 * per GPU, held from the library's first use on that GPU until the process
 * ends (its address is looked up once per device).  Maps with ncomp*ny*nx*16
 * bytes + 4.2 MB above 64 MiB (e.g. I,Q,U above 1024 x 1024) are rejected
 * with MM_EINVAL.  The call must be made with the scan's device current.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (other threads, other streams) race and give wrong spectra.
 * Unlike mm_map_spectra it does not touch the scan's preconditioner scratch,
 * so it may run while a preconditioner apply of the same handle is in flight.
 * Calls no hipMalloc, hipFree or other allocating routine. */
mm_status mm_map_spectra_noalloc(mm_scan scan, const double* x, double pixel_arcmin, double dell,
                                 int32_t nbins, double* spectra /*[host]*/, double* counts /*[host]*/,
                                 void* stream);

/* Delayed A-norm error estimate of PCG (footnote of the Results section,
 * with r_j.z_j for ||r_j||^2 under a preconditioner): est[k] =
 * sum_{j=k}^{k+delay-1} alpha_j rho_j for k = 0..n-delay, an estimate of
 * ||x_k - x||_A^2.  alpha, rho: [host] n scalars as returned in
 * mm_pcg_result; est: [host] max(n - delay + 1, 0) entries.  Host only. */
mm_status mm_anorm_error_estimate(const double* alpha /*[host]*/, const double* rho /*[host]*/,
                                  int32_t n, int32_t delay, double* est /*[host]*/);

/* Error of a spectrum in cosmic-variance units (the Results section's
 * convergence measure): err[c][b] = |c_iter[c][b] - c_input[c][b]| / sigma_b
 * with sigma_b = c_input[c][b] sqrt(2 / N_b), N_b = counts[b] / 2 (a real
 * map's independent modes); NaN where the bin is empty or c_input <= 0.
 * All arrays [host], [ncomp][nbins] (counts [nbins]).  Host only. */
mm_status mm_spectrum_cv_error(const double* c_iter, const double* c_input, const double* counts,
                               int32_t ncomp, int32_t nbins, double* err /*[host]*/);

/* The CG step at which a per-bin error first reaches `threshold` once the
 * errors of n recorded steps are averaged over consecutive blocks of `block`
 * steps: linear interpolation between the centres of the last block above
 * and the first block at or below the threshold (the first block's centre if
 * that one is already below).  *found = 0 (and *step unchanged) if no block
 * reaches it.  steps, errors: [host] n values.  Host only. */
mm_status mm_cv_crossing_step(const double* steps, const double* errors, int32_t n,
                              double threshold, int32_t block, double* step /*[host]*/,
                              int32_t* found /*[host]*/);

/* Diagnostics of a scan handle. */
typedef struct {
  int32_t n_active;         /* active pixels */
  int32_t ref_pixel;        /* circulant reference pixel id, -1 if not built */
  int32_t n_floored;        /* eigenvalues raised by the circulant floor */
  int32_t det_group;        /* detectors per pipeline group in use */
  int32_t fft_m1, fft_m2;   /* four-step split in use (m1 = 1: one-pass kernel) */
  int32_t fft_cols;         /* columns per pass-1/3 block (0: one-pass kernel) */
  int32_t single_pass;      /* 1 if each detector's filter runs in one kernel */
  int32_t csr;              /* how P^T runs: 0 atomic scatter; 1 per-pixel gather
                               through a per-sample index; 2 per-pixel gather through
                               runs of consecutive samples (stored pointing, groups
                               of at most 2^28 samples) */
  size_t  workspace_bytes;  /* bytes used */
  int32_t gather_weights;   /* how the P^T gather gets the I,Q,U weights: 0 float32
                               pairs stored with the index, 1 computed from the
                               boresight model, 2 stored as 4-byte angles (stored
                               weights of unit norm on the float32 and bfloat16
                               paths; decoded to within 1e-7), -1 no gather or I only */
  int32_t pass1_pointing;   /* what pass 1 reads for the pointing: 0 stored pixels and
                               weights (or I only, or a timestream), 1 the boresight
                               model, 2 stored pixels and time-major angles, 3 the
                               chunk-coded pixels and angles (pointing_code) */
  double  t_build_s;        /* wall time of the last mm_build_precon on this handle */
} mm_scan_info;

mm_status mm_get_info(mm_scan scan, mm_scan_info* out /*[host]*/);

/* Copies the active-pixel mask (int32, 1 = active) into dst [ny][nx]. */
mm_status mm_get_mask(mm_scan scan, int32_t* dst, void* stream);

/* Per-stage device timing for benchmarks: while enabled, every launch of a
 * timed stage is bracketed by two HIP events recorded on the stream it runs
 * on; mm_profile_read waits for them, returns the summed durations and
 * resets.  Stages: 0 one-pass filter kernel, 1 four-step pass 1 (gather +
 * column FFTs), 2 pass 2 (row FFTs + 1/N(f) + inverse row FFTs), 3 pass 3
 * (inverse column FFTs, + atomic scatter without the pixel index), 4 one
 * whole A-apply or right-hand side, 5 one preconditioner apply, 6 the
 * per-pixel gather of P^T, 7 the cross-detector projection of correlated
 * noise (pass 2 then times its unpack and its filtered repack).
 * samples[i] counts the timestream samples (stages 0-4, 6, 7) or map entries
 * (stage 5) the launches processed. */
typedef struct {
  int32_t n_stages;
  double  ms[8];
  int64_t launches[8];
  int64_t samples[8];
} mm_profile;

mm_status mm_profile_enable(mm_scan scan, int32_t enable);
/* Restricts the timing to the stages whose bit (1 << stage) is set in mask
 * (default: every stage); the others record no events, so a benchmark can
 * time one kernel without the event overhead on the rest.  Kept across
 * mm_profile_enable calls. */
mm_status mm_profile_stages(mm_scan scan, uint32_t mask);
mm_status mm_profile_read(mm_scan scan, mm_profile* out /*[host]*/);

/* Thread-local message describing the last non-OK status ("" if none). */
const char* mm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MM_H */

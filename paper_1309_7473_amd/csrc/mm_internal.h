// Internal host-side state of a scan handle and the launch helpers shared by
// the translation units of libmm.so.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/mm.h"
#include "pointing.h"

namespace mm {

constexpr int kNT = 256;         // threads per block of the timestream kernels
constexpr int kE = 32;           // complex elements per thread in LDS FFTs
constexpr int kMapE = 16;        // ... in the float64 map FFTs
constexpr int kHistCap = 65536;  // PCG history entries kept on the device
constexpr int kMaxPartials = 1024;
constexpr int kProfStages = 8;   // see mm_profile in mm.h
constexpr int kSpecBlocks = 256;   // blocks of the map-spectra binning
constexpr int kSpecMaxBins = 512;  // multipole bins of mm_map_spectra
// device scratch of mm_map_spectra_noalloc (one static array per device)
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
constexpr int kPtcLog = 6;
constexpr int kPtcChunk = 1 << kPtcLog;   // samples per chunk of the chunk-coded pointing
constexpr int kProfSingle = 0, kProfPass1 = 1, kProfPass2 = 2, kProfPass3 = 3, kProfApplyA = 4,
              kProfPrecon = 5, kProfReduce = 6, kProfCorr = 7;

void set_error(const std::string& msg);
mm_status fail(mm_status st, const std::string& msg);
mm_status hip_check(hipError_t e, const char* what);

#define MM_HIP(call)                                          \
  do {                                                        \
    hipError_t _e = (call);                                   \
    if (_e != hipSuccess) return ::mm::hip_check(_e, #call);  \
  } while (0)

// Device-resident PCG scalars.
struct PcgDev {
  double rho;      // r_k . z_k
  double ps;       // p . A p
  double rr;       // ||r||^2
  double bb;       // ||b||^2
  double rz;       // new r.z
  double alpha, beta;
  double tol2;
  double true_rr;  // ||b - A x||^2 over the active entries (true-residual check)
  int iters;
  int done;
  int breakdown;
  int cf;          // reductions in compensated float32 pairs
  int flex;        // Polak-Ribiere beta = -alpha (s.z') / rho
};

// Offsets of the sub-buffers inside the caller's workspace.
struct Layout {
  size_t tod;        // pipeline scratch: G * M complex (0 bytes if single pass)
  size_t tw;         // Stockham table, Lmax complex
  size_t tw2;        // W_{2 M2}^k2 table, M2 complex (four-step)
  size_t tw_m1;      // M1 complex (W_M1^m, mixed-radix columns)
  size_t int_;       // ndet * (M+1) float: 1/N(f) in four-step order
  size_t wn_hi, wn_lo;
  size_t gmap;       // (npix + 1) * 4 real (gather map; entry npix is zero)
  size_t acc;        // npix * 4 double (scatter accumulator)
  size_t detw;       // ndet double
  size_t hits;       // npix double (hit counts, accumulated in f64)
  size_t bb, bj;     // npix * 6 double: binned / Jacobi blocks (packed symmetric)
  size_t binv_b, binv_j, siginv;  // npix * 6 double
  size_t sigma;      // npix * 6 double: B^(1/2) (packed symmetric)
  size_t mask;       // npix int32
  size_t kinv;       // npix * nc*nc complex double
  size_t planes;     // ncomp^2 * npix complex double (FFT scratch, probe q planes)
  size_t probe;      // nc*nc*npix double
  size_t tw_map;     // max(ny,nx) complex double
  size_t vec;        // 5 CG vectors of nc*npix double (r, z, p, s, tmp)
  size_t partials;   // kMaxPartials * 4 double
  size_t pcg;        // PcgDev
  size_t hist;       // 3 * (kHistCap+1) double
  size_t misc;       // small ints / doubles (ref key, floor count, lambda max)
  size_t spec;       // map-spectra partials and result (kSpecBlocks+1) * kSpecMaxBins * 4 double
  size_t corr_edges; // corr_nbins + 1 int32 (copied from the descriptor)
  size_t corr_bin;   // M + 1 int16: frequency bin of each four-step slot
  size_t corr_t;     // corr_rank * M complex: low-rank projections of the spectra
  size_t csr_cnt;    // ngroups * npix int32 (counts, then fill cursors)
  size_t csr_off;    // ngroups * (npix+1) int32
  size_t csr_soff;   // run-length index with angle-coded weights: ngroups * (npix+1)
                     // int32 offsets of each pixel's samples in the pixel-major angles
  size_t csr_idx;    // ngroups * G * n int32 (group-relative sample index), or
                     // uint32 run entries (first sample << 4 | length)
  size_t csr_w;      // ngroups * G * n float2 (cos 2psi, sin 2psi), or uint32 angles
  size_t ang_tab;    // 256 float2: (cos, sin)(2 pi k / 256)
  size_t ang_t;      // ndet * n uint32: the weights as angles, time-major (pass 1)
  size_t ptc_h;      // ndet * n/kPtcChunk int4: chunk-coded pointing, per chunk
                     // (smallest on-map pixel, angle base, angle slope, 0)
  size_t ptc;        // ndet * n uint32: chunk-coded pointing, per sample
                     // (pixel - smallest | (angle - base - slope * i) << 16)
  size_t bore_f, bore_a, det_f, det_a;   // float32 copies of the boresight model
  size_t total;
};

struct Plan {
  bool f64;
  bool bf16;         // bfloat16 timestream and pass buffers (float math)
  bool acc32;        // compensated float32 accumulation (MM_ACC_F32X2)
  int corr_rank;     // > 0: inter-detector correlated N^-1 (one group, split pass 2)
  int corr_nbins;
  bool single;       // whole detector filtered in one kernel
  bool csr;          // P^T by per-pixel gather (else atomic scatter)
  bool otf;          // pointing computed from the boresight model
  bool csr_w;        // the gather has stored weights (in the index, or time-major
                     // beside the pointing with the run-length index)
  bool rle;          // the pixel-major index holds runs of consecutive samples
  bool ptc;          // pass 1 may read the chunk-coded pointing (sized in the layout)
  uint32_t mix_code; // mixed-radix stage code of M (one kernel) or M1 (four-step); 0: power of two
  int M1;            // four-step column length (2^logM1 unless mixed)
  int logn, logM;    // n = 2^logn samples, M = n/2 packed complex
  int logM1, logM2;  // four-step split
  int logC;          // columns per pass-1/3 block
  int G;             // detectors per group
  int logLmax;       // Stockham table length
  int logS;          // two-level table split for W_n
  int logMapL;       // map FFT table length
};

struct Profiler;
template <typename T>
struct Cx;

struct ScanImpl {
  mm_scan_desc d;
  int nc, ny, nx, ndet, npix;
  int64_t n;
  Plan plan;
  Layout lay;
  char* ws;
  int ref_pixel = -1;
  int n_floored = 0;
  double t_build_s = 0.0;   // wall time of the last mm_build_precon
  int n_active = 0;
  bool circ_built = false;
  bool csr_ang = false;       // the index's weights are stored as fixed-point angles
  bool ang_t_ready = false;   // pass 1 reads the time-major angles (SRC 3)
  bool ptc_ready = false;     // pass 1 reads the chunk-coded pointing (SRC 5)
  bool rle_pa = false;        // the run-length gather reads pixel-major angles
  double* fuse_y = nullptr;   // output map the last group's gather may write directly
  bool fused_y = false;       // set when it did (the epilogue is then skipped)
  bool bore_fast = false;     // pass 1 evaluates the boresight model in float32 (SRC 4)
  bool tiled_built = false;   // tiled preconditioner
  int tiled_T = 0;
  char* tiled_ws = nullptr;   // caller-owned workspace of the tiled preconditioner
  int circ_sym = 1;
  int maxdyn_lds = 65536;
  Profiler* prof = nullptr;
  uint32_t prof_mask = ~0u;   // stages timed while profiling is enabled
  bool capturing = false;   // launches are being recorded into a graph
  mm_learned learned = nullptr;

  template <typename P>
  P* at(size_t off) const { return reinterpret_cast<P*>(ws + off); }
};

// The boresight model of a scan (pointers null for stored pointing).
inline Bore scan_bore(const ScanImpl* s) {
  Bore b;
  if (s->plan.otf) {
    b.b = s->d.bore;
    b.det = s->d.det_off;
  }
  b.logn = s->plan.logn;
  b.ndet = s->ndet;
  b.ny = s->ny;
  b.nx = s->nx;
  return b;
}

// ---- launchers implemented across the .hip files -------------------------
mm_status plan_and_layout(const mm_scan_desc* d, Plan* plan, Layout* lay);
mm_status upload_tables(ScanImpl* s, hipStream_t st);
mm_status filter_pipeline(ScanImpl* s, int src /*0 gather x, 1 timestream*/,
                          const void* tod, const double* x, double* y, hipStream_t st);
mm_status binned_setup(ScanImpl* s, hipStream_t st);
mm_status csr_setup(ScanImpl* s, hipStream_t st);
mm_status bore_setup(ScanImpl* s, hipStream_t st);
mm_status permute_inverse_spectrum(ScanImpl* s, hipStream_t st);
mm_status binned_apply(ScanImpl* s, int jacobi, const double* r, double* z, hipStream_t st);
mm_status circulant_build(ScanImpl* s, const mm_precon_opts* o, hipStream_t st);
mm_status circulant_apply(ScanImpl* s, const double* r, double* z, hipStream_t st);
bool tiled_size_ok(const ScanImpl* s, int T);
size_t tiled_workspace_bytes(const ScanImpl* s, int T);
mm_status tiled_build(ScanImpl* s, const mm_precon_opts* o, hipStream_t st);
mm_status tiled_apply(ScanImpl* s, const double* r, double* z, hipStream_t st);
// 2-D FFT of nplanes complex double [ny][nx] planes in place (unnormalised)
mm_status map_fft(ScanImpl* s, Cx<double>* planes, int nplanes, bool inv, hipStream_t st);
mm_status precon_judge(ScanImpl* s, const int32_t* cand, int n, const double* b, double* x,
                       const mm_pcg_opts* o, mm_pcg_result* res, int32_t* chosen, hipStream_t st);
mm_status map_spectra_noalloc(ScanImpl* s, const double* x, double pixel_arcmin, double dell,
                              int nbins, double* spectra, double* counts, hipStream_t st);
mm_status map_spectra(ScanImpl* s, const double* x, double pixel_arcmin, double dell, int nbins,
                      double* spectra, double* counts, hipStream_t st);
mm_status pcg_solve(ScanImpl* s, int precon, const double* b, double* x,
                    const mm_pcg_opts* o, mm_pcg_result* res, hipStream_t st);
mm_status pcg_solve_batch(ScanImpl* const* scans, int n, int precon, const double* const* b,
                          double* const* x, const mm_pcg_opts* o, mm_pcg_result* res,
                          mm_status* status, hipStream_t st);
mm_status fill_zero(void* p, size_t bytes, hipStream_t st);
mm_status apply_precon(ScanImpl* s, int precon, const double* r, double* z, hipStream_t st);
void prof_begin(ScanImpl* s, hipStream_t st, hipEvent_t* tok, int stage);
void prof_end(ScanImpl* s, hipStream_t st, hipEvent_t tok, int stage, int64_t samples);
mm_status profile_enable(ScanImpl* s, int enable);
mm_status profile_stages(ScanImpl* s, uint32_t mask);
mm_status profile_read(ScanImpl* s, mm_profile* out);
void profile_free(ScanImpl* s);
// learned correction (learned.hip)
mm_status learned_apply(ScanImpl* s, const double* r, double* z, hipStream_t st);
mm_status learned_make_pair(ScanImpl* s, const double* xf, const double* xk, float* rw, float* t,
                            float* e2, hipStream_t st);
size_t learned_workspace_bytes(int nc, int ny, int nx, int batch);
mm_status learned_create(int nc, int ny, int nx, int batch, void* ws, size_t ws_bytes,
                         const float* w1, const float* w2, hipStream_t st, mm_learned* out);
void learned_destroy(mm_learned h);
mm_status learned_get(mm_learned h, float* w1, float* w2);
mm_status learned_check(mm_learned h, int nc, int ny, int nx);
mm_status learned_train(mm_learned h, const float* rw, const float* t, const float* e2,
                        int64_t npairs, const mm_train_opts* o, double* loss_hist, hipStream_t st);
mm_status learned_loss(mm_learned h, const float* rw, const float* t, const float* e2,
                       int64_t npairs, double* loss, hipStream_t st);
mm_status learned_forward(mm_learned h, const float* x, int B, float* y, float* a1, float* a2,
                          float* a3, hipStream_t st);
mm_status learned_grad(mm_learned h, const float* rw, const float* t, const float* e2, int B,
                       double* loss, float* g1, float* g2, hipStream_t st);

}  // namespace mm

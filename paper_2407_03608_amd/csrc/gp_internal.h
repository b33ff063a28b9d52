// Internal declarations shared by the gpnufft translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gpnufft.h"
#include "gp_rules.h"

namespace gp {

// ------------------------------------------------------------------ errors --
void set_error(const std::string& msg);
void clear_error();

#define GP_HIP(call)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::gp::Error{GP_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define GP_CHECK_LAUNCH() GP_HIP(hipGetLastError())

// --------------------------------------------------------- device buffers --
// Stream-ordered device memory: alloc takes memory in the order of stream st
// (usable by work queued on st afterwards) and release returns it in the order
// of the stream it was taken on, so neither waits for the device.  The memory
// comes from the device's pool, which keeps released memory for reuse instead
// of returning it to the driver.  Work on other streams that uses a buffer
// must be complete before the buffer is released.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t s = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void alloc(size_t b, hipStream_t st);
  void release();
  template <class T> T* as() const { return static_cast<T*>(p); }
};
// Pinned host blocks of kCgScalars doubles, kept for reuse (freeing pinned
// memory would wait for the whole device).
double* pinned_scalars_get();
void pinned_scalars_put(double* h);

// One batched pass of 1-D FFTs along one axis of a strided array:
// element (o, pos, c) of the input lives at in[o*in_os + i*inner + c] where
// i = (pos - in_start) mod L and i < n_in (other positions are zero); the
// output keeps positions out_start .. out_start + n_out - 1 (mod L) at
// out[o*out_os + i*inner + c].  sign = -1 forward, +1 inverse (unnormalised).
// tw4 != null applies the four-step twiddle exp(sign 2 pi i pos*o / L4) on load
// (tw4_at_load = 1) or on store (0); tw4 holds exp(-2 pi i k / L4), k < L4.
struct FftPass {
  int L;
  int64_t n_outer;
  int64_t inner;
  int64_t in_os, out_os;
  int n_in, in_start, n_out, out_start;
  int sign;
  const void* tw4 = nullptr;
  int64_t L4 = 0;
  int tw4_at_load = 1;
  // Transform (o, c), o < n_outer, c < inner, reads element i at
  //   in + o in_os + (c / cp) in_cs + (c % cp) in_cs1 + (i / ip) in_es + (i % ip) in_es1
  // and writes element i at the same form over out (cp, ip = 1 or 2: pairs of
  // transforms or of elements interleaved).  es = 0 means inner (the sequence
  // runs across the batch), cs = 0 means 1.
  int64_t in_es = 0, in_cs = 0, out_es = 0, out_cs = 0;
  int in_cp = 1, in_ip = 1, out_cp = 1, out_ip = 1;
  int64_t in_cs1 = 0, in_es1 = 0, out_cs1 = 0, out_es1 = 0;
};
void fft_pass(int fp64, const FftPass& p, const void* in, void* out, const void* twiddles,
              hipStream_t s);

// ---------------------------------------------------------- point records --
// A point set sorted into the spreading tiles.  Each point carries its first
// window cell per dimension and a row of `rs` T values: the d*w window values
// psi(cell + q - g) followed by the nkp weights w_k(x) of eq:Wk.
struct Records {
  int64_t n = 0;
  int rs = 0;                 // row length of pw (T elements)
  DevBuf perm;                // int32  [n] sorted -> caller index
  DevBuf cell;                // int32  [d][n] first window cell in the active box
  DevBuf pw;                  // T      [n][rs] window values and w_k
  DevBuf bin_start;           // int32  [n_bins + 1]
  // Work lists that split crowded tiles into point chunks (built with the
  // bin sort; see build_work_lists):
  //  sp_work  int4 {tile, lo, hi, slot}: spread the tile's source points
  //           [lo, hi) (positions in the tile's source sequence) into the
  //           grid (slot < 0) or into partial tile `slot`
  //  sp_red   int4 {tile, slot0, count, 0}: grid tile = sum of its partials,
  //           added in slot order
  //  in_work  int4 {bin, p_lo, p_hi, 0}: interpolate sorted points [p_lo, p_hi)
  //  in_work2 int4 {super-bin, lo, hi, 0} (d >= 2): interpolate positions
  //           [lo, hi) of the points of a 2x2(x1) block of bins (its two bin rows
  //           in order, each a contiguous range of the sorted points)
  DevBuf sp_work, sp_red, in_work, in_work2, part;
  int64_t n_sp_work = 0, n_sp_red = 0, n_in_work = 0, n_in_work2 = 0, n_slots = 0;
  // Sub-tile spreading (fp32 grids, d >= 2; see build_spread_lists): sub-tiles
  // of sub_st^d cells, numbered bin * (sub-tiles per bin) + sub, and for each
  // the points whose window reaches it, in visiting order:
  //  sub_off   int64 [n_sub + 1]   start of each sub-tile's list
  //  sub_list  int2 [sub_off[n_sub]]  {sorted index, first window cell
  //            relative to the sub-tile origin - (w - 1), 8 bits per dimension}
  DevBuf sub_off, sub_list;
  int64_t n_sub = 0;
  int sub_st = 0;
};

// ------------------------------------------------------------------- plan --
// A plan: its numbers (PlanRules, chosen on the host) and its device data.
// Step-3 tile of orthant points in 2-D: the mode kernels visit these tiles in
// order of their distance from the origin, so the points in flight at any time
// lie in one annulus and share a narrow band of the radial table.
constexpr int kModeTileX = 64, kModeTileY = 4;

struct Plan : PlanRules {
  int64_t n = 0;
  double eta = 0;
  int device = 0;             // HIP device current when the plan was built
  // device data
  hipStream_t stream = nullptr;
  Records rec;                // the training points, bin-sorted
  DevBuf nodes_d;             // double [nk] sigma_k
  DevBuf bary_d;              // double [nk] barycentric weights
  DevBuf gtab;                // T [nt][nk][M+1]: C_kj * exp(-tau_kj n^2) for dim 0
  DevBuf etab;                // T [nt][nk][M+1]: exp(-tau_kj n^2) for dims >= 1
  DevBuf vtd;                 // T [nt] v~_j
  int step3 = 0;              // 0: radial precomputed A, 1: direct t-sum, 2: low-rank radial A
  DevBuf lr_off;              // int64 [a_rows + 1]: start of each row's factors in atab (step3 = 2)
  int lr_rank_max = 0;        // largest rank over the rows (step3 = 2)
  double lr_rank_mean = 0;
  int spread_mode = GP_SPREAD_OWNER;  // resolved gp_opts.spread (never GP_SPREAD_AUTO)
  int interp_mode = 0;        // 0 default, 1 cache gather, 2 per-bin LDS tiles
  DevBuf atab;                // T [a_rows][nkp(nkp+1)/2] upper triangle of A_k'k(|n|^2)
  DevBuf rowidx;              // int32 [d M^2 + 1]: |n|^2 -> row (d >= 2)
  DevBuf mode_tiles;          // int32: 2-D orthant tiles of kModeTileX x kModeTileY points,
                              // nearest the origin first (step3 = 0)
  int64_t mode_ntx = 0;       // tiles along n_0
  DevBuf dec;                 // T [d][M+1] 1/psi^(2 pi n / nf_r)
  DevBuf tw[3];               // FFT twiddles per distinct length (T complex)
  DevBuf tw4;                 // four-step twiddles (1-D, T complex, length nf)
  DevBuf gridA, gridB, gridB2, gridC;
  int64_t grid_elems[4] = {0, 0, 0, 0};  // complex elements per grid pair of A, B, B2, C
  // The grids the matvec kernels read and write: the plan's own (one set), or
  // the batched grids of a multi-vector application, `nsets` consecutive sets
  // of npair pairs each.  Spreading and interpolation work on set `cur`; the
  // FFT passes and step 3 on all sets at once.
  struct GridView {
    void *A = nullptr, *B = nullptr, *B2 = nullptr, *C = nullptr;
    int nsets = 1;
    int cur = 0;
  } gv;
  DevBuf mA, mB, mB2, mC;     // batched grids for up to m_cap vectors (allocated on first use)
  int m_cap = 0;
  DevBuf vec;                 // fp64 scratch vectors for matvec / CG (sorted order)
  // CG reductions (allocated once per plan): per-block partial sums, the
  // scalar slots of the solver and a pinned host mirror of those slots
  DevBuf cg_part;             // double [kCgBlocks]
  DevBuf cg_S;                // double [kCgScalars]
  double* cg_hS = nullptr;    // pinned host, kCgScalars
  size_t device_bytes = 0;
  // optional per-phase event timing
  bool timing = false;
  struct Ev {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Ev> events;
  std::vector<hipEvent_t> pool;
  ~Plan();
};

enum Phase {
  PH_SPREAD = 0,
  PH_FFT_FWD0 = 1,
  PH_MODE = 4,
  PH_FFT_INV2 = 5,
  PH_INTERP = 8,
  PH_CG = 9,
  PH_COUNT = 10
};
extern const char* const kPhaseNames[PH_COUNT];

// Brackets a group of launches with HIP events when the plan times itself.
struct PhaseScope {
  Plan* P;
  int phase;
  hipEvent_t b = nullptr;
  PhaseScope(Plan* p, int ph);
  ~PhaseScope();
};

// plan.hip
int build_plan(int d, int64_t n, const double* pts, const double* sigma, const double* l,
               double nu, double eta, double tol, const gp_opts* opts, Plan* P, bool query_only,
               size_t* bytes_out);

// nufft.hip: y = K~ x (+ eta^2 x) with x, y fp64 in SORTED order on the plan stream.
void matvec_sorted(Plan* P, const double* x_sorted, double* y_sorted, int add_noise);
// The same for m vectors at once (x, y: m consecutive sorted-order vectors of
// length n), sharing each FFT pass and the step-3 table reads: the result for
// every vector has the same bits as matvec_sorted gives it.  Uses batched
// grids for up to `m` vectors (allocated on first use; GP_ENOMEM if they do not fit).
void matvec_multi_sorted(Plan* P, int m, const double* x_sorted, double* y_sorted, int add_noise);
// Largest m for which the batched grids fit in half of the free device memory.
int multi_capacity(Plan* P, int want);
// Evaluate the type-2 + combine step at arbitrary mapped targets after a forward
// pass of x_sorted; used by the posterior mean.
void posterior_sorted(Plan* P, const double* x_sorted, int64_t m, const double* tpts,
                      const double* tsig, const double* tl, double* mu);
// gather / scatter between caller and sorted order
// K~ between record sets of one plan (same grid and box): forward_from puts
// the grids of sum_i xs_i delta(x - x_i) over the points of R (sorted order)
// through spreading, both FFTs and the mode mixing; interp_from_grid then
// writes ys = K~(points of R', those points) xs for any record set R'.
void forward_from(Plan* P, const Records& R, const double* xs);
void interp_from_grid(Plan* P, const Records& R, double* ys);
// Kernel arguments of the spreading and interpolation kernels for one point
// set (training points or targets) and one chunk of grid pairs.
struct NuArgs {
  int64_t n;
  int nk, npair, w;
  double beta;
  int tile[3], nbins[3], na[3];
  int64_t gstride[3];  // element strides of the active grid (dim 0 contiguous)
  int64_t pair_stride;
  int64_t grid_off;
  int g0, gc, nsrc;
  int slot_pairs;  // grid pairs per partial tile slot (min(8, npair))
  double eta2;
  int add_noise, first_chunk;
};
NuArgs nu_args(const Plan* P, const Records& R);
// Release the plan's device memory in the order of stream st from now on
// (after its previous stream has been synchronised).
void retag_plan_stream(Plan* P, hipStream_t st);
// Grid A (spread output, interpolation input) of the current vector set.
void* grid_a_current(const Plan* P);

// Spreading in d >= 2 works on sub-tiles of spread_sub_side(P)^d cells, one
// wavefront each, from per-sub-tile point lists built once per plan
// (gp_spread.hip); other plans spread whole tiles.
int spread_sub_side(const Plan* P);  // 0 when the plan spreads whole tiles
inline bool spread_uses_sub_tiles(const Plan* P) { return spread_sub_side(P) > 0; }
// Device bytes of the sub-tile lists, bounded before the points are sorted.
size_t spread_list_bound_bytes(const Plan* P, int64_t n);
void build_spread_lists(Plan* P, Records& R);
void spread_sub_launch(Plan* P, const Records& R, const double* xs);
// out[0..n) = exclusive prefix sums of the counts in[0..n) (device arrays, on
// stream s); *total = their sum, read back to the host.
void exclusive_scan_counts(const int* in, int64_t n, int64_t* out, hipStream_t s, int64_t* total);
void build_records_into(Plan* P, int64_t n, const double* pts, const double* sig,
                        const double* l, Records& R, int* out_of_box);
void gather_sorted(Plan* P, const double* x_user, double* x_sorted);
void scatter_user(Plan* P, const double* x_sorted, double* x_user);

// cg.hip
// Device memory a CG solve reduces into: `part` holds one partial sum per
// reduction block (kCgBlocks), `S` the solver's scalar slots (kCgScalars);
// hS is a pinned host mirror of S, or null (reads then go through a
// synchronous copy to the stack).
constexpr int kCgBlocks = 512;
constexpr int kCgScalars = 16;
struct CgScratch {
  double* part;
  double* S;
  double* hS;
};
CgScratch plan_cg_scratch(Plan* P);
// x = 0 on the plan's stream (a kernel, not a memset)
void zero_sorted(Plan* P, double* x);
int cg_solve_sorted_with(Plan* P, const CgScratch& sc, const double* b, double* x, bool x_zero,
                         double tol, int max_iter, int replace_every, int* iters, double* rel_res);
int cg_solve_sorted(Plan* P, const double* b, double* x, bool x_zero, double tol, int max_iter,
                    int replace_every, int* iters, double* rel_res);
double dot_sorted(Plan* P, const double* a, const double* b, int64_t n);
// CG for m right-hand sides in lockstep, sharing each operator application
// (b, x: m consecutive sorted vectors, x = 0 on entry; iters, rel: host, m)
int cg_multi_sorted(Plan* P, int m, const double* b, double* x, double tol, int max_iter,
                    int* iters, double* rel);
// block CG (shared Krylov space) for 1..16 right-hand sides, same layout
int cg_block_sorted(Plan* P, int m, const double* b, double* x, double tol, int max_iter,
                    int* iters, double* rel);
// refinement with two plans on the same points, vectors in caller order (capi.hip)
int cg_refined_user(Plan* Pi, Plan* Po, const double* y, double* alpha, double tol,
                    double inner_tol, int max_iter, int max_refine, int replace_every,
                    int* iters, double* rel, int* passes);
// ||b - (K~ + eta^2 I) x||^2 and ||b||^2 (sorted order)
void residual_norms(Plan* P, const double* b, const double* x, double* rr, double* bb);

}  // namespace gp

struct gp_plan_s {
  gp::Plan P;
};

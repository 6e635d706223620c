// Internal declarations of the esnufft library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <cstdint>
#include <vector>

#include "../../include/esnufft.h"

namespace esn {

constexpr int kMaxW = 16;        // widest kernel supported (eps ~ 1e-15)
constexpr int kMaxDim = 3;

// ---- host plan math (params.cpp) ----
bool width_from_eps(double eps, int* w_out);
int64_t next_smooth235(int64_t n);
int64_t fine_size(int64_t N, double sigma, int w);
void gauss_legendre_positive(int p, std::vector<double>* nodes,
                             std::vector<double>* weights);
int quad_nodes_for_width(int w);

// Point storage codes: how a sorted point's fine-grid coordinates t in [0, n)
// are kept.  Each sorted point is one record holding its coordinates and its
// original index (the permutation entry):
//   kPtsFixed32: 16 bytes {uint32 q[3], int32 perm}, q = t * 2^F unsigned fixed
//                point (F = 32 - ceil(log2 n) fraction bits), used by
//                single-precision plans on grids up to 8192;
//   kPtsF64:     32 bytes {double t[3], int32 perm, pad}.
// Unused dimensions hold 0.
enum { kPtsFixed32 = 1, kPtsF64 = 2 };
inline int pts_record_bytes(int code) { return code == kPtsFixed32 ? 16 : 32; }

// Everything a spread/interp kernel needs about the geometry and the sorted
// points.  Passed by value.
// Stage events of one setpts or execute of a debug plan (types 1 and 2).
// kind 1: setpts (e0 start, e1 end); kind 2 / 3: single-chunk execute in the
// type 1 / type 2 direction (e5 start, e0 .. e3 around the stage before the
// FFT, the FFT and the stage after it, e4 end); kind 4: values computed at the
// call (multi-chunk execute).
struct TimingRec {
  int kind = 0;
  hipEvent_t e[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  esn_stats vals{};
};
constexpr int kTimingRing = 256;

// Piecewise polynomial kernel (Sec. 5.3): degree w + kPolyExtra per interval.
constexpr int kPolyExtra = 3;

struct GeomArgs {
  int64_t n[3];          // fine grid per dim (1 for unused dims)
  int b[3];              // bin size per dim (1 for unused dims)
  int nb[3];             // bins per dim
  int fbits[3];          // fixed-point fraction bits per dim
  int pts_code;          // kPtsFixed32 or kPtsF64
  double beta;           // ES shape parameter
  int64_t M;             // number of points
  int ntr;               // transforms in this launch
  int64_t cstride;       // elements between transforms in c (= M)
  int64_t gstride;       // elements between transforms in the grid
  const unsigned char* pts;  // sorted point records (see kPtsFixed32 / kPtsF64)
  const int32_t* sub_bin;    // subproblem -> bin
  const int32_t* sub_start;  // subproblem -> first sorted position
  const int32_t* sub_len;    // subproblem -> number of points
  int nsub;                  // number of subproblems
  // piecewise polynomial kernel table [w][w + kPolyExtra + 1] in the plan's
  // precision (esn_kernel_poly), or null: exp and sqrt at every weight
  const void* ktab;
};

// ---- kernel launchers (kernels_*.hip) ----
// All return hipSuccess or the launch error.
hipError_t launch_fseries(int w, double beta, const double* d_nodes,
                          const double* d_weights, int nquad, int64_t nf, int64_t N,
                          double* d_out, hipStream_t s);

hipError_t launch_deconv(int prec, int dim, const int64_t* N, const int64_t* nf,
                         int modeord, int ntr, const void* grid, int64_t gstride,
                         void* f, int64_t fstride, const double* const* pf,
                         hipStream_t s);
hipError_t launch_amplify(int prec, int dim, const int64_t* N, const int64_t* nf,
                          int modeord, int ntr, void* grid, int64_t gstride,
                          const void* f, int64_t fstride, const double* const* pf,
                          hipStream_t s);

// Sorting / binning (kernels_sort.hip).
//
// Points are counted per fine-grid cell.  Cells are numbered bin-major: the
// key of a cell is bin * cpb + local, cpb = b0 b1 b2 cells per bin, with the
// local index z-fastest in 3D (local = lz + b2 (lx + b0 ly)), so that the
// cells of one (x, y) column of a bin are consecutive keys and
// column = key / b2.  In 2D local = lx + b0 ly, in 1D local = lx.
struct SortArgs {
  int dim;
  int64_t M;
  int coord_prec;           // ESN_SINGLE / ESN_DOUBLE
  const void* x[3];         // caller's coordinates
  int64_t n[3];
  double inv_n[3];          // 1 / n
  double scale[3];          // n / 2pi
  double span[3], pow2f[3]; // n 2^fbits and 2^fbits (fixed-point coordinates)
  int b[3], nb[3], fbits[3];
  int bpow2;                // every b[m] is 2^bshift[m]
  int bshift[3];
  int pts_code;
  int chkbnds;
  int w;                    // kernel width (decides each point's window cell)
  int blocked;              // 3D cell order by 2 x 2 column blocks (even b[0], b[1])
  int blocked2d;            // 2D cell order by blocked2d x blocked2d blocks (4 or 8; 0: row-major)
  uint32_t* key;            // [M] cell key of each point (counting sort)
  int32_t* slot;            // [M] rank of the point within its cell (counting sort)
  int32_t* count;           // [ncells + 1] points per cell (counting sort)
  const int32_t* sstart;    // [ncells + 1] first sorted position of a cell (counting sort)
  unsigned char* pts;       // [M] point records (counting sort: sorted; no sort:
                            // input order)
  int32_t* flags;           // [1]: bit0 NaN/inf, bit1 out of range
};
// Point records written unsorted (no binning).
hipError_t launch_encode_unsorted(const SortArgs& a, hipStream_t s);
// Radix sort (large point sets): least-significant digit first, digits of
// dbits <= kRsMaxDigitBits bits, passes <= kRsMaxPasses.
constexpr int kRsMaxDigitBits = 8;
constexpr int kRsMaxPasses = 4;
struct RsortArgs {
  int passes = 0, dbits = 0, ntiles = 0;
  int64_t tp = 0;               // points per tile
  int vec4 = 0;                 // coordinate arrays aligned for 4-point vector loads
  int32_t* count = nullptr;     // [2^dbits][ntiles] digit counts per tile
  int32_t* offset = nullptr;    // [2^dbits][ntiles] their exclusive scan
};
// Passes of a key of key_bits bits (*dbits: bits per digit).
int radix_digits(int key_bits, int* dbits);
// Points per tile of a pass.
int64_t radix_tile_points(int rec_bytes);
// Scratch bytes of radix_sort_points for M points.
size_t radix_scratch_bytes(int64_t M, int key_bits, int rec_bytes);
// Stable sort of the points of a (a.M, a.x; coordinate checks into
// a.flags[0]) by key (keys below 2^key_bits): records in key order into
// out_rec (M records), the sorted keys into scratch (*sorted_keys).
hipError_t radix_sort_points(const SortArgs& a, int key_bits, unsigned char* out_rec,
                             void* scratch, size_t scratch_bytes, uint32_t** sorted_keys,
                             hipStream_t s);
// key[i] and perm[i] of every stored record pts[i], i < a.M (a.dim, a.n, a.b,
// a.nb, a.fbits, a.pts_code, a.w, a.blocked set).
hipError_t launch_record_keys(const SortArgs& a, const unsigned char* pts, uint32_t* key,
                              int32_t* perm, hipStream_t s);
// Counting sort: count each point into its cell (the count before the
// increment is its slot), then, after an exclusive scan of the counts, store
// its record at start[cell] + slot.
hipError_t launch_bin_count(const SortArgs& a, hipStream_t s);
hipError_t launch_scatter(const SortArgs& a, hipStream_t s);
// bstart[b] = sstart[b * cpb] for b = 0 .. nbins.
hipError_t launch_bin_starts(const int32_t* sstart, int64_t cpb, int64_t nbins, int32_t* bstart,
                             hipStream_t s);
// endpos[b] = one past the last sorted position of bin b = key / cpb for each
// bin with points (endpos zeroed by the caller, nbins entries).
hipError_t launch_bin_ends(const uint32_t* skey, int64_t M, int cpb, int32_t* endpos,
                           hipStream_t s);
// Subproblems of every bin: runs of at most maxsub of its points, in bin order.
// With endpos (bin ends from launch_bin_ends) the bin starts are written to
// bstart[0 .. nbins]; without it bstart must hold them.  nsub gets nbins
// per-bin counts, tiles 3 bin_tiles(nbins) ints of per-tile partials; the
// sub_* arrays must hold every subproblem (at most min(nbins, M) + M / maxsub).
// totals[0] = number of subproblems, totals[1] = bins with points.
int64_t bin_tiles(int64_t nbins);
hipError_t launch_bin_subproblems(const int32_t* endpos, int32_t* bstart, int64_t nbins,
                                  int64_t M, int maxsub, int32_t* nsub, int32_t* tiles,
                                  int32_t* sub_bin, int32_t* sub_start, int32_t* sub_len,
                                  int32_t* totals, hipStream_t s);
// Exclusive scan of n int32 values (in -> out, may not alias); tmp must hold
// scan_tmp_elems(n) int32.
int64_t scan_tmp_elems(int64_t n);
hipError_t exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n,
                              int32_t* tmp, hipStream_t s);
hipError_t launch_iota_i32(int32_t* p, int64_t n, hipStream_t s);

// Spread / interp (kernels_spread.hip, kernels_interp.hip).
// method 1: LDS tile per subproblem (grid = nsub workgroups);
// method 2: one thread per point with global atomics / direct gathers.
hipError_t launch_spread(int method, int prec, int dim, int w, const GeomArgs& g,
                         int nsub, int block, size_t lds_bytes, const void* c,
                         void* grid, hipStream_t s);
hipError_t launch_interp(int method, int prec, int dim, int w, const GeomArgs& g,
                         int nsub, int block, size_t lds_bytes, const void* grid,
                         void* c, hipStream_t s);
// Matrix-core spreading / interpolation (kernels_mfma.hip): 3D, single
// precision, w <= 7, fixed-point coordinates, one transform per launch; one
// wave per subproblem.
hipError_t launch_spread_mfma(int w, const GeomArgs& g, int nsub, const void* c, void* grid,
                              hipStream_t s);
hipError_t launch_interp_mfma(int w, const GeomArgs& g, int nsub, const void* grid, void* c,
                              hipStream_t s);
size_t mfma_spread_lds_bytes(int w, const int* b);
size_t mfma_interp_lds_bytes(const int* b);
// Matrix-core spreading / interpolation in 2D (kernels_mfma2d.hip): single or
// double precision, w <= 13, bins of whole 4 x 4 blocks of window cells, g.ntr
// transforms per launch sharing the staged weights; one wave per subproblem.
hipError_t launch_spread_mfma2d(int prec, int w, const GeomArgs& g, int nsub, const void* c,
                                void* grid, hipStream_t s);
hipError_t launch_interp_mfma2d(int prec, int w, const GeomArgs& g, int nsub, const void* grid,
                                void* c, hipStream_t s);
size_t mfma2d_lds_bytes(int prec, int w, const int* b, int ntr, bool spread);
// Block of window cells of the 2D matrix-core kernels at width w (8 for w <= 9, else 4).
inline int mfma2d_block(int w) { return w <= 9 ? 8 : 4; }

// LDS bytes one subproblem tile needs for ntr transforms (with the spreading
// kernel's per-point staging when staging is true).
size_t tile_lds_bytes(int prec, int dim, int w, const int* b, int ntr, bool staging = true);

// ---- type 3 (kernels_type3.hip, type3.cpp) ----
// Chebyshev coefficients per dimension of the type 3 correction sum (see
// T3Args::cheb).
constexpr int kT3Cheb = 24;
// Per-point (sources) or per-target work of Sec. 3.3 on n values.
struct T3Args {
  int dim, isign, w;
  int64_t n;
  double x0[3], s0[3];          // centres of the sources and the targets
  double inv_gam[3];            // 1 / gamma: sources x'' = (x - x0) / gamma
  double hgam[3];               // h gamma: targets s'' = h gamma (s - s0)
  double* out[3];               // rescaled coordinates (FP64, n each)
  // The correction sum g(u) = sum_q w_q phi(z_q) cos(u z_q) at u = (w/2) s''
  // as sum_k cheb[m][k] T_k(u^2 cscale[m] - 1) over |u| <= U_m, the largest
  // |u| of the targets (cscale = 2 / U_m^2; 0 and cheb = {g(0), 0, ...} when
  // U_m = 0).
  double cheb[3][kT3Cheb];
  double cscale[3];
};
// Coordinate arrays (device) whose bounds one launch finds.
struct MinMaxSets {
  const void* x[6];
  int64_t n[6];
  int count;
};
// Bounds of each array i < a.count into out[2 i] (min), out[2 i + 1] (max; NaN
// if any value is NaN or infinite); part holds
// 2 a.count t3_minmax_blocks(max n) doubles of per-block partials.
int t3_minmax_blocks(int64_t n);
hipError_t launch_minmax(const MinMaxSets& a, int coord_prec, double* part, double* out,
                         hipStream_t s);
// Rescaled sources into a.out and prephase factors exp(isign i s0.(x - x0)) into pre.
hipError_t launch_t3_sources(const T3Args& a, int coord_prec, int prec, const void* const* x,
                             void* pre, hipStream_t s);
// Rescaled targets into a.out and per-target factors (correction of step 3 times
// the postphase exp(isign i s.x0)) into post.
hipError_t launch_t3_targets(const T3Args& a, int coord_prec, int prec, const void* const* sx,
                             void* post, hipStream_t s);
// out[t][i] = in[t][i] * fac[i], i < n, t < ntr (complex of precision prec).
hipError_t launch_cmul(int prec, const void* in, const void* fac, void* out, int64_t n, int ntr,
                       hipStream_t s);

// ---- Toeplitz form of the normal operator (kernels_toeplitz.hip, toeplitz.cpp) ----
struct ToepArgs {
  int64_t N[3];    // modes per dim (1 for unused dims)
  int64_t L[3];    // doubled grid 2 N (1 for unused dims)
  int modeord;     // order of the caller's mode arrays
};
hipError_t launch_fill_ones(int prec, void* c, int64_t n, hipStream_t s);
hipError_t launch_scale(int prec, void* v, int64_t n, double s, hipStream_t st);
// grid (L) = the caller's modes f at positions k + floor(N/2), zeros elsewhere
hipError_t launch_toep_pad(const ToepArgs& a, int prec, const void* f, void* grid, hipStream_t s);
// f = the modes back out of grid positions k + floor(N/2)
hipError_t launch_toep_extract(const ToepArgs& a, int prec, const void* grid, void* f,
                               hipStream_t s);

// Plan creation behind esn_makeplan for types 1 and 2; spread_only: no FFT
// plans and no fine grid (a plan that sorts points and spreads into caller
// grids, esn_spread).
int make_plan(int type, int dim, const int64_t* nmodes, int isign, int ntransf, double eps,
              int prec, esn_plan* out, const esn_opts* opts, void* stream, bool spread_only);
// Stage times of a debug plan's latest setpts and execute (waits for them).
int plan_stats(esn_plan p, esn_stats* o);
// setpts behind esn_setpts (ext_scratch null) and esn_setpts_noalloc
// (ext_scratch: the sort's scratch of ext_bytes bytes; radix sort, no
// allocation, the plan must already hold room for M points).
int setpts_impl(esn_plan p, int64_t M, int coord_prec, const void* const* xs, void* ext_scratch,
                size_t ext_bytes);
// Type 3 plans (type3.cpp).
int t3_makeplan(int dim, int isign, int ntransf, double eps, int prec, esn_plan* out,
                const esn_opts* opts, void* stream);
int t3_execute(esn_plan p, void* c, void* f);
void t3_destroy(esn_plan p);

// ---- rocFFT wrapper (fft.cpp) ----
// In 3D only the x columns that hold modes (k1 mod n1 for k1 in I_N1, two
// runs) need the FFTs along y and z: after the x pass of a type 1 transform the
// other columns are never read, and before the x pass of a type 2 transform
// they are zero.  Such a plan runs one batched x pass and, per transform and
// kept run, a 2D (y, z) FFT batched over the run's columns.
// One pass of column FFTs (kernels_fft.hip): DFTs of length L along a stride
// of estride elements, for blocks of 32 neighbouring x columns of each of
// nplanes planes (pstride apart) and each transform (tstride apart).  Column
// blocks 0 .. chunks_a - 1 come first, then the blocks from chunk_b0 on;
// likewise planes 0 .. planes_a - 1, then the planes from plane_b0 on.
constexpr int kColWidth = 32;
struct ColFFTArgs {
  int64_t estride = 0, pstride = 0, tstride = 0, nplanes = 0;
  int64_t planes_a = 0, plane_b0 = 0;
  // kept points of a DFT (masked or mode-array ends): j < keep_lo or
  // j >= L - keep_hi
  int64_t keep_lo = 0, keep_hi = 0;
  int chunks_a = 0, chunk_b0 = 0;
  int sign = 1;
};
// Mode arrays and correction factors of a z pass that reads p_k f_k (type 2)
// or writes f_k = p_k b^_k (type 1) itself.
struct ColModes {
  float2* f = nullptr;                  // transform t at f + t fstride
  int64_t fstride = 0;
  int64_t N[3] = {1, 1, 1};             // modes per dim
  int64_t n0 = 0, n1 = 0;               // fine-grid x and y lengths
  const double* pf[3] = {nullptr, nullptr, nullptr};   // p_k per dim
  int modeord = 0;
};
// in_mode / out_mode: 0 the grid, 1 the grid at the kept points only, 2 the
// mode arrays (z pass).
hipError_t launch_fft_cols(float2* data, int L, const ColFFTArgs& a, const double2* tw,
                           int nchunks, int ntr, int in_mode, int out_mode, const ColModes& cm,
                           hipStream_t s);
hipError_t launch_zero_cols(float2* data, int64_t n0, int64_t rows, int64_t x0, int64_t x1,
                            int ntr, int64_t tstride, hipStream_t s);
// Lengths the column FFTs take: 2^a 3^b 5^c with a >= 5, up to 512.
bool fft_cols_supported(int64_t L);

struct FFTPlan {
  rocfft_plan plan = nullptr;          // the whole transform, or the x pass
  rocfft_plan yz[2] = {nullptr, nullptr};   // (y, z) FFTs of the kept x runs
  int64_t yz_off[2] = {0, 0};          // first column of each kept run
  int nyz = 0;                         // kept runs (0: not pruned)
  int batch = 0;                       // transforms
  int64_t grid = 0;                    // elements per transform
  int elem = 8;                        // bytes per complex element
  int x_first = 1;                     // type 1: x pass first; type 2: last
  // pruned single-precision transforms whose y and z lengths the column FFTs
  // take: the kept columns' y and z passes run as column FFTs
  int cols = 0;
  int modes = 0;                       // the correction folds into the z pass
  int padded = 0;                      // zero-padded transform (fft_make_padded)
  ColFFTArgs cy, cz;
  ColFFTArgs cy_keep, cz_keep;         // the same, keeping the points that hold modes
  int64_t nx = 0;                      // x length
  int ly = 0, lz = 0, nchunks = 0;
  double2* d_tw = nullptr;             // twiddles of length ly, then of length lz
  hipStream_t stream = nullptr;
  rocfft_execution_info info = nullptr;
  void* work = nullptr;
  size_t work_bytes = 0;
};
// nmodes: N per dim, for the kept x runs of a 3D transform; type selects the
// pass order.
int fft_make(FFTPlan* p, int dim, const int64_t* nf, const int64_t* nmodes, int type, int batch,
             int prec, int sign, hipStream_t s);
int fft_exec(FFTPlan* p, void* data);
// With the correction folded into the column passes (p->cols): type 1
// (x_first) transforms the spread grid and writes f = p_k b^_k for the modes;
// type 2 reads the modes f with their factors p_k and leaves the transformed
// grid (no amplification before it).  Layout of f as for deconv / amplify.
int fft_exec_modes(FFTPlan* p, void* grid, void* f, const ColModes& cm);
void fft_destroy(FFTPlan* p);
// Transform of a 3D grid of lengths L whose input (input_padded = 1) or
// needed output (0) lies in [0, N) per dimension, the rest of the input being
// zero: single precision with column-FFT lengths skips the y and z passes of
// the columns outside; otherwise the full transform.  One transform per call.
int fft_make_padded(FFTPlan* p, int dim, const int64_t* L, const int64_t* N, int prec, int sign,
                    hipStream_t s);
int fft_exec_padded(FFTPlan* p, void* data, int input_padded);
// Move an FFT plan's work to another stream.
void fft_trim(FFTPlan* p);
int fft_ensure_work(FFTPlan* p);
int fft_set_stream(FFTPlan* p, hipStream_t s);

// Move a plan (and its rocFFT execution info) to another stream.  The caller
// makes sure no work of the plan is pending on the old stream.
int plan_set_stream(esn_plan p, hipStream_t s);
// Give back the memory a plan needs only while it works (fine grid, FFT work
// buffers, sorted points and sort scratch); the plan keeps its parameters,
// tables and FFT plans, needs a setpts before its next execute, and makes
// the buffers again then.  For plans kept idle in a cache.  Returns the
// plan's remaining device bytes.
int64_t plan_trim(esn_plan p);
// Device bytes a plan of this shape would hold with M points (an estimate used
// for admission before the plan exists; rocFFT's work buffer is taken as one
// fine grid).
int64_t plan_estimate_bytes(int type, int dim, const int64_t* nmodes, double eps, int prec,
                            int64_t M);

}  // namespace esn

// The plan object behind esn_plan.
struct esn_plan_s {
  int type, dim, isign, ntransf, prec;
  int64_t N[3], nf[3];
  double eps;
  esn_params par;
  esn_opts opts;
  hipStream_t stream;
  int device;
  int warn;                      // status to return for eps warnings

  // correction factors p_k per dim, FP64, k = 0..floor(N/2)
  double* d_pf[3] = {nullptr, nullptr, nullptr};
  // fine grid(s): chunk * nf1 nf2 nf3 complex
  void* d_grid = nullptr;
  int chunk = 1;                 // transforms per fused launch
  esn::FFTPlan fft;
  esn::FFTPlan fft_tail;         // plan for the last, shorter chunk (if any)
  // the opposite transform direction (esn_execute_adjoint): FFTs of sign
  // -isign, made on its first call; its transforms per launch and last chunk
  esn::FFTPlan fft_adj;
  esn::FFTPlan fft_adj_tail;
  int adj_chunk = 0, adj_tail = 0;
  int tail = 0;

  // binning geometry
  int bin[3] = {1, 1, 1};
  int nb[3] = {1, 1, 1};
  int64_t nbins = 1;
  int maxsub = 1024;
  int spread_method = 1, interp_method = 1;
  int kerevalmeth = 1;           // 1 exp and sqrt, 2 polynomial table (d_ktab)
  void* d_ktab = nullptr;        // [w][w + kPolyExtra + 1] in the plan precision
  int block = 256;
  int pts_code = esn::kPtsFixed32;
  int fbits[3] = {0, 0, 0};

  // points
  int64_t M = -1;                // -1: no points yet
  int64_t cap_M = 0;
  unsigned char* d_pts = nullptr;   // [M] sorted point records
  uint32_t* d_ckey = nullptr;    // [M] cell keys (counting sort)
  void* d_rscratch = nullptr;    // radix sort scratch (radix_scratch_bytes(cap_M))
  size_t rscratch_bytes = 0;
  int key_bits = 0;              // bits of the largest cell key
  int64_t ncells = 0;            // bins * cells per bin
  int64_t cap_count = 0;         // points the counting sort buffers hold
  int32_t* d_slot = nullptr;     // [M] counting sort: slot within the cell
  int32_t* d_count = nullptr;    // [ncells + 1] counting sort: points per cell
  int32_t* d_sstart = nullptr;   // [ncells + 1] counting sort: first position of a cell
  int32_t* d_cell_scan_tmp = nullptr;   // scan scratch over the cells
  int last_sort = 0;             // method of the last setpts (2 radix, 3 counting)
  int32_t* d_bend = nullptr;     // [nbins] one past a bin's last sorted position (0: empty)
  int32_t* d_bstart = nullptr;   // [nbins + 1] first sorted position of a bin
  int32_t* d_nsub = nullptr;
  int32_t* d_tiles = nullptr;    // [3 bin_tiles(nbins)] per-tile partials
  int32_t* d_flags = nullptr;
  int32_t* d_sub_bin = nullptr;
  int32_t* d_sub_start = nullptr;
  int32_t* d_sub_len = nullptr;
  int64_t cap_sub = 0;
  int nsub = 0;
  int nbins_nonempty = 0;
  int32_t* h_pinned = nullptr;   // small pinned host buffer for read-backs
  bool spread_only = false;      // no FFT plans or fine grid: sorts and spreads only

  // type 3 (Sec. 3.3): a spread-only type 1 plan spreads the prephased,
  // rescaled sources onto the type 3 fine grid; a type 2 plan with that grid
  // as its modes (FFT order) evaluates it at the rescaled targets
  esn_plan_s* t3_spread = nullptr;
  esn_plan_s* t3_inner = nullptr;
  int64_t t3_N = -1;             // targets (-1: no points yet)
  int64_t t3_n[3] = {1, 1, 1};   // type 3 fine grid n_i, eq. (ng)
  double t3_x0[3] = {0, 0, 0}, t3_s0[3] = {0, 0, 0}, t3_gam[3] = {1, 1, 1};
  void* d_t3_pre = nullptr;      // [M] prephase factors (complex, plan precision)
  void* d_t3_post = nullptr;     // [N] correction times postphase
  void* d_t3_grid = nullptr;     // [ntransf][n1 n2 n3] spread grid = inner modes
  void* d_t3_c = nullptr;        // [ntransf][M] prephased strengths
  double* d_t3_xy = nullptr;     // [2][3][cap] rescaled sources, targets (setpts scratch)
  hipStream_t t3_side = nullptr; // second stream: the targets' sort beside the sources'
  hipEvent_t t3_ready = nullptr; // rescaled targets written
  std::vector<double> t3_zq, t3_wphi;   // quadrature nodes, weights * phi at them
  double* d_t3_mm = nullptr;     // min/max partials
  double* h_t3_mm = nullptr;     // pinned copy of the partials
  int64_t t3_cap_M = 0, t3_cap_N = 0, t3_cap_grid = 0, t3_cap_xy = 0;

  // debug timing.  Type 3 plans time their steps with ev and keep the values
  // in stats.  Types 1 and 2 record the stage events of each setpts and
  // execute in a ring and read them only when asked (esn_get_stats), so that
  // timing adds no host synchronisation to the calls.
  hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  esn_stats stats{};
  std::vector<esn::TimingRec> ring;
  int64_t ring_count = 0;        // calls recorded so far
  int64_t device_bytes = 0;
  std::vector<std::pair<void*, size_t>> allocs;   // live device allocations
};

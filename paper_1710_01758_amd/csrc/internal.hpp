// Internal device-side descriptors and kernel launchers (not part of the ABI).
#pragma once

#include "common.hpp"

namespace pics {

// Columns per column tile: 16 up to length 320 (128-byte row segments), 4 at
// 512 (a single large slice then still gives the chip enough workgroups), 8
// at 1024.
constexpr int kColT = 16;
__host__ __device__ constexpr int col_tile(int m) { return m >= 1024 ? 8 : m >= 512 ? 4 : kColT; }
// The fused operator's alternative tile widths (autotuner candidates besides
// col_tile(m)), two per length, each giving workgroups of 64 to 1024 threads:
// 8 and 32 at the lengths carried by 8 threads per column (64, 128, 224), 8
// and 4 at those with 16 (192, 256, 320), 8 and 2 at 512, 4 and 2 at 1024.
__host__ __device__ constexpr int apply_tile_alt(int m, int k) {
  return m >= 1024 ? (k == 0 ? 4 : 2)
       : m >= 512  ? (k == 0 ? 8 : 2)
       : (m == 64 || m == 128 || m == 224) ? (k == 0 ? 8 : 32)
                                            : (k == 0 ? 8 : 4);
}
constexpr int kRowRR = 16;    // rows per row tile
constexpr int kPartMax = 256;  // partial sums per slice per reduction (n / col_tile(m) <= 256)

// reduction slots (per slice: kSlots x kPartMax doubles)
enum PartSlot { P_SIGMA = 0, P_RR = 1, P_BB = 2, P_RHO0 = 3, P_RHO1 = 4, P_AUX = 5, kSlots = 6 };

// Tile of workgroup b (column tiles, wavelet tiles).  Workgroups go to the 8 XCDs in turn (linear
// id mod 8) and each XCD has its own L2, so each XCD is given a run of
// adjacent tiles: cache lines shared by neighbouring tiles (the operator's
// halo columns, tiles narrower than a line) are then fetched into one L2.
__device__ __forceinline__ int xcd_tile(int b, int ntiles) {
  if (ntiles & 7) return b;
  return (b & 7) * (ntiles >> 3) + (b >> 3);
}

struct SliceDev {
  int m, n, nc, mask_kind;  // mask_kind: 0 = line mask uint8[m], 1 = 2D uint8[m][n]
  int wavelet, levels;      // 0 none, 1 haar, 2 db4
  float mu, lam, gam;
  int ctiles;  // column tiles of the line-mask operator (n / its tile width): sigma partials per solve
  long long img;   // element offset of the slice in packed image-shaped buffers
  long long coil;  // element offset in packed coil-shaped buffers [nc][m][n]
  long long mask;  // byte offset in the packed mask buffer
  long long aux;   // offset of the slice's (n / col_tile(m)) x m FP64 coil-power partials
};

// Per-slice PCG control block; lives in device memory.
struct PcgState {
  int it_a;    // completed x/r updates (written by the update kernel only)
  int it_r;    // copy of it_a taken by the apply kernel (read by the update kernel)
  int done;    // 1 once converged, broken down or stopped
  int status;  // 1 converged, 0 running / max iterations, < 0 error code
  int iters;   // iterations at exit
  int maxit;   // per-slice iteration cap for this solve
  double relres;
};

// Device pointers shared by the kernels (passed by value).
struct Ws {
  const SliceDev* sl;
  const int* group;       // launch grid.y -> slice index
  const float2* sens;     // packed [nc][m][n] per slice
  const uint8_t* mask;    // packed masks
  const float2* tw;       // packed twiddle tables
  const float* kinv;      // 1 / (k m n) per pixel (circulant / learned)
  const float* jac;       // 1 / diag(A) per pixel (Jacobi)
  double* part;           // [nslices][kSlots][kPartMax]
  PcgState* st;           // [nslices]
};

__device__ __forceinline__ double* part_ptr(double* part, int s, int slot) {
  return part + ((long long)s * kSlots + slot) * kPartMax;
}
__device__ __forceinline__ double part_sum(const double* p, int count) {
  double acc = 0.0;
  for (int i = 0; i < count; ++i) acc += p[i];
  return acc;
}

// preconditioner kinds (same values as the ABI)
enum { PK_NONE = 0, PK_JACOBI = 1, PK_CIRC = 2, PK_LEARNED = 3 };

// column-tile apply modes
enum { CA_APPLY = 0, CA_PCG = 1 };
// apply phases: one fused pass, or per-coil-group partial data terms + finish
enum { AP_FUSED = 0, AP_PART = 1, AP_FIN = 2 };
// apply term flags
enum { TERM_DATA = 1, TERM_TV = 2, TERM_GAMMA = 4, TERM_ALL = 7 };
// row-tile update modes
enum { RU_SETUP = 0, RU_UPDATE = 1 };

struct Launch {
  hipStream_t stream;
  int m, n;          // common size of the slices in this group
  int count;         // slices in this group
  const int* group;  // device array of slice indices
};

// Arguments of one wavelet pass (see k_sb.hip).
struct WaveArgs {
  int level, inverse, pass, last, mode;  // mode 0: store, 1: SB shrink (analysis) / right-hand side (synthesis)
  int fresh;                             // shrink: the Bregman variables start at zero (not read)
  const float2* in;
  float2* out;
  float2* coef;
  float2* bw;
  float2* uw;
  const float2* tvr;  // synthesis, mode 1: g + lam (D_x^H u_x + D_y^H u_y), from the level-0 analysis
  float2* rhs;
};

// Fused TV shrink/update carried by the level-0 wavelet analysis.
// Image-domain outer update fused into the shrink kernels (level 0):
// mode 1: q = b - r (= A x after the solve that produced r);
// mode 2: also g <- g + g1 - A_data x with A_data x = q - lam L x - gam x.
// End-of-solve record of a fixed-budget solve (graph replays), carried by the
// first shrink kernel after the solve: every slice's stop test, then its
// iteration count and status stored at row *counter of the history; then the
// counter advances.  counter == nullptr: no record.
struct SolveRecord {
  int* iters;
  int* status;
  int* counter;
  double tol;
  int nslices;
};

struct OuterArgs {
  int mode;
  const float2* b;
  const float2* r;
  float2* q;
  float2* g;
  const float2* g1;
  SolveRecord rec;
};

// Fused TV shrink/update of the level-0 analysis.  It leaves the TV part of
// the next right-hand side, tvr = g + lam (D_x^H u_x + D_y^H u_y) (g after the
// outer update), instead of u_x and u_y.
// The Bregman variables b_x, b_y are read from bxi, byi and written to bx, by
// (two buffers used in turn: a workgroup reads the old b on its neighbours'
// pixels, which they overwrite in the same launch).
struct TvArgs {
  int enabled;
  const float2* bxi;
  const float2* byi;
  float2* bx;
  float2* by;
  float2* tvr;
  OuterArgs outer;
  int fresh;  // b_x, b_y start at zero (not read)
};

struct Simple {
  hipStream_t stream;
  int nslices;
  long long max_pixels;
};

bool fft_size_supported(int N);

// ---- FFT-path launchers (k_fft_ops.hip)
// ngroups > 1 splits the coil loop over up to that many workgroups per tile
// (partial data terms in dpart[group][image-packed], stride dstride elements)
// and adds them in a second pass.  ncmax > 0: the group's largest coil count;
// a slice then takes only as many workgroups as keep each at or below
// ceil(ncmax / ngroups) coils (0: every slice takes ngroups).
// tile: the operator's column-tile width (0 = col_tile(m); else one of
// apply_tile_alt(m, 0 / 1), with no coil split).
hipError_t launch_col_apply(const Launch& L, const Ws& w, int mode, int terms, int pk, double tol,
                            const float2* xin, const float2* zsrc, const float2* pold, float2* pn, float2* out,
                            int ngroups = 1, float2* dpart = nullptr, long long dstride = 0, int tile = 0,
                            int ncmax = 0);
// tile widths launch_col_apply accepts for an m x n slice
bool apply_tile_ok(int m, int n, int tile);
// RU_SETUP also resets the slices' PCG state (iteration limit maxit, or
// maxit_ps[slice] when given)
hipError_t launch_row_update(const Launch& L, const Ws& w, int mode, int pk, const float2* b, const float2* q,
                             float2* x, float2* r, const float2* pn, float2* p, float2* t, int maxit = 0,
                             const int* maxit_ps = nullptr);
hipError_t launch_col_precond(const Launch& L, const Ws& w, int use_state, int check, double tol, float2* t,
                              float2* x);
hipError_t launch_row_z(const Launch& L, const Ws& w, const float2* t, const float2* r, float2* z);
hipError_t launch_row_fft(const Launch& L, const Ws& w, int inverse, int ncoil_mode, const float2* in, float2* out);
hipError_t launch_col_fft(const Launch& L, const Ws& w, int inverse, const float2* in, float2* out);
hipError_t launch_col_sb_init(const Launch& L, const Ws& w, const float2* coil_rows, float2* g1, float2* g,
                              float2* rhs, float2* x);
hipError_t launch_col_coil_power(const Launch& L, const Ws& w, double* pbar, float* energy);
hipError_t launch_col_coil_energy(const Launch& L, const Ws& w, const float2* coil_rows, float* energy);

// ---- 2D sampling masks (k_mask2d.hip)
// the system operator as row / column / row passes through the coil buffer
// `coil` (coil-shaped); modes and arguments as launch_col_apply
hipError_t launch_apply2d(const Launch& L, const Ws& w, int mode, int terms, int pk, double tol, const float2* xin,
                          const float2* zsrc, const float2* pold, float2* pn, float2* out, float2* coil);
hipError_t launch_col_power2d(const Launch& L, const Ws& w, const float2* coil_rows, float* P, float* energy);
hipError_t launch_corr_prep(const Simple& S, const Ws& w, const float* P, float2* a, float2* b);
hipError_t launch_corr_mul(const Simple& S, const Ws& w, float2* a, const float2* b);
hipError_t launch_build_k2d(const Simple& S, const Ws& w, const float2* a, const float* corr, const float* energy,
                            float* kraw, float* kinv, float* jac, int* bad);

// ---- coil compression (k_coils.hip); scratch: the coil workspace viewed as
// double2, per slice at coil offset / 2; eigenvalues to the P_AUX slot
hipError_t launch_coil_compress(const Simple& S, const Ws& w, const float2* ksp, const float2* sens, int nvirt,
                                double2* scratch, float2* ksp_out, float2* sens_out);

// ---- 3D extension (k_volume.hip); V voxels, nc coil volumes back to back
constexpr int kVolDotBlocks = 256;
hipError_t launch3_coil_mul(hipStream_t st, const float2* S, const float2* x, float2* out, int nc, long long V);
hipError_t launch3_mask_scale(hipStream_t st, float2* buf, const uint8_t* mask, int nc, long long V, float scale);
hipError_t launch3_accumulate(hipStream_t st, const float2* S, const float2* buf, const float2* x, float2* y, int nc,
                              int p, int m, int n, float mu, float lam, float gam, int data);
hipError_t launch3_power(hipStream_t st, const float2* buf, float* P, int nc, long long V);
hipError_t launch3_corr_prep(hipStream_t st, const uint8_t* mask, const float* P, float2* a, float2* b, long long V);
hipError_t launch3_corr_mul(hipStream_t st, float2* a, const float2* b, long long V);
hipError_t launch3_build_k(hipStream_t st, const float2* a, float* kraw, float* kinv, int* bad, int p, int m, int n,
                           double mu, double lam, double gam);
hipError_t launch3_scale(hipStream_t st, float2* buf, const float* s, long long V);
// operator passes for masks constant along x over the chunk of columns
// x0 .. x0 + X - 1 (X a multiple of col_tile(m) dividing n; the chunk
// workspace `coil` is [nc][p][m][X]; see k_volume.hip)
hipError_t launch3_col_sp(hipStream_t st, const float2* S, const float2* x, float2* coil, const float2* tw, int nc,
                          int p, int m, int n, int x0, int X);
hipError_t launch3_col_z(hipStream_t st, float2* coil, const uint8_t* mask, const float2* tw, int nc, int p, int m,
                         int n, int x0, int X, float scale);
hipError_t launch3_col_acc(hipStream_t st, const float2* S, const float2* coil, const float2* x, float2* y,
                           const float2* tw, int nc, int p, int m, int n, float mu, float lam, float gam, int data,
                           int x0, int X);
hipError_t launch3_xconst(hipStream_t st, const uint8_t* mask, long long rows, int n, int* flag);
// scal[idx] = Re(a^H b) in FP64 (partials in part[slot][kVolDotBlocks], fixed-order sum)
hipError_t launch3_dot(hipStream_t st, const float2* a, const float2* b, long long V, double* part, int slot,
                       double* scal, int idx);
hipError_t launch3_residual(hipStream_t st, const float2* b, const float2* q, float2* r, long long V);
hipError_t launch3_update_xr(hipStream_t st, float2* x, float2* r, const float2* p, const float2* q, const double* scal,
                             int irho, int isig, long long V);
hipError_t launch3_update_p(hipStream_t st, float2* p, const float2* z, const double* scal, int inew, int iold,
                            long long V);
// packed twiddle tables tw[tw_offset(N) + k] = exp(-2 pi i k / N) (host, FP64 rounded)
void fill_twiddles(float2* tw_host);

// ---- per-pixel kernels (k_sb.hip)
hipError_t launch_pcg_check(hipStream_t st, const Ws& w, int nslices, double tol, int setup, float2* x);
hipError_t launch_tv_shrink(const Simple& S, const Ws& w, int only_nowavelet, int fresh, const OuterArgs& oa,
                            const float2* x, const float2* bxi, const float2* byi,
                            float2* bx, float2* by, float2* ux, float2* uy, float2* bw, float2* uw);
hipError_t launch_rhs_nowavelet(const Simple& S, const Ws& w, const float2* g, const float2* ux, const float2* uy,
                                const float2* uw, float2* rhs);
// one wavelet level (analysis or synthesis per a.inverse); `tiles` = max over
// slices of the level's 16 x 16 coefficient tiles
hipError_t launch_wavelet(const Simple& S, const Ws& w, const WaveArgs& a, const TvArgs& tv, int tiles);
int wavelet_tiles(int m, int n, int level);
hipError_t launch_build_k(const Simple& S, const Ws& w, double* pbar, const float* corr, float* kraw,
                          float* kinv, float* jac, int* bad);
hipError_t launch_fill(hipStream_t st, float2* p, long long count, float2 v);
hipError_t launch_add_gamma(const Simple& S, const Ws& w, const float2* wx, const float2* x, float2* y);
// end-of-solve stop test of every slice, then the per-slice iteration count
// and status recorded at history row *counter (the counter advances)
hipError_t launch_set_int(hipStream_t st, int* p, int v);

}  // namespace pics

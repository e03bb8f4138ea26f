// Per-pixel kernels around the FFT passes: PCG control, the Split Bregman
// shrink/update steps (Algorithm 1, steps 6-11), the periodised orthonormal
// wavelet passes and the circulant spectrum assembly.
//
// Launch shape: grid (blocks, nslices), a grid-stride loop over one slice's
// pixels per grid.y, so slices of different sizes share one launch.
#include <algorithm>

#include "internal.hpp"

namespace pics {

// Lowpass filters.  Haar: 1/sqrt(2) (1, 1).  Daubechies-4 (8 taps, 4 vanishing
// moments, extremal phase), listed as in Daubechies, Ten Lectures on Wavelets,
// Table 6.1 (N = 4), normalised to sum sqrt(2).  Highpass g[t] = (-1)^t h[K-1-t].
__constant__ float c_haar[2] = {0.70710678118654752f, 0.70710678118654752f};
__constant__ float c_db4[8] = {0.2303778133088964f,  0.7148465705529154f,  0.6308807679298587f,
                               -0.0279837694168599f, -0.1870348117190931f, 0.0308413818355607f,
                               0.0328830116668852f,  -0.0105974017850690f};

__device__ __forceinline__ float2 shrink(float2 v, float thr) {
  const float a = sqrtf(v.x * v.x + v.y * v.y);
  if (!(a > thr)) return make_float2(0.f, 0.f);
  const float s = 1.0f - thr / a;
  return make_float2(v.x * s, v.y * s);
}

// ------------------------------------------------------------ PCG control

// Stop test of one slice: converged (status 1), iteration limit (0), or, at
// the set-up, a zero right-hand side (converged, x = 0; returns true).
__device__ __forceinline__ bool slice_stop_test(const Ws& w, int s, double tol, int setup) {
  const SliceDev& sd = w.sl[s];
  PcgState* st = w.st + s;
  if (st->done) return false;
  const int nrt = sd.m / kRowRR;
  const double rr = part_sum(part_ptr(w.part, s, P_RR), nrt);
  const double bb = part_sum(part_ptr(w.part, s, P_BB), nrt);
  int status = -100;
  bool zero_x = false;
  if (setup && bb == 0.0) {
    zero_x = true;
    status = 1;
  } else if (rr <= tol * tol * bb) {
    status = 1;
  } else if (st->it_a >= st->maxit) {
    status = 0;
  }
  if (status != -100) {
    st->done = 1;
    st->status = status;
    st->iters = st->it_a;
    st->relres = bb > 0.0 ? sqrt(rr / bb) : 0.0;
  }
  return zero_x;
}

// Stop test at the set-up and at host polling points.  A zero right-hand side
// gives x = 0 with no iterations.
__global__ __launch_bounds__(256) void k_pcg_check(Ws w, double tol, int setup, float2* __restrict__ x) {
  const int s = blockIdx.x;
  const SliceDev sd = w.sl[s];
  __shared__ int zero_x;
  if (threadIdx.x == 0) zero_x = slice_stop_test(w, s, tol, setup) ? 1 : 0;
  __syncthreads();
  if (zero_x) {
    const long long np = (long long)sd.m * sd.n;
    for (long long p = threadIdx.x; p < np; p += blockDim.x) x[sd.img + p] = make_float2(0.f, 0.f);
  }
}

// End of a fixed-budget solve (graph replays), run by workgroup (0, 0) of the
// first shrink kernel after the solve (nothing reads the PCG control blocks
// between the solve and the next set-up).
__device__ void record_solve(const Ws& w, const SolveRecord& rc) {
  __shared__ int row;
  if (threadIdx.x == 0) row = *rc.counter;
  __syncthreads();
  for (int s = threadIdx.x; s < rc.nslices; s += blockDim.x) {
    slice_stop_test(w, s, rc.tol, 0);
    rc.iters[(long long)row * rc.nslices + s] = w.st[s].iters;
    rc.status[(long long)row * rc.nslices + s] = w.st[s].status;
  }
  if (threadIdx.x == 0) *rc.counter = row + 1;
}

__global__ void k_set_int(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// --------------------------------------------------- outer update (fused)
// After a PCG solve, A x = b - r exactly in exact arithmetic (r is the
// solver's residual), so the next solve's A x0 and the data term of the outer
// update (Algorithm 1 steps 13-15, image-domain form)
//   A_data x = A x - lam (D_x^H D_x + D_y^H D_y) x - gam x
// need no further operator application.  lap = 4 x - (four neighbours).
__device__ __forceinline__ float2 outer_at(const SliceDev& sd, const OuterArgs& oa, long long pp, float2 xc,
                                           float2 lap, float2 bv, float2 rv, float2 gv, float2 g1v) {
  const float2 ax = csub(bv, rv);
  oa.q[pp] = ax;
  if (oa.mode == 2) {
    const float2 ad = make_float2(ax.x - sd.lam * lap.x - sd.gam * xc.x, ax.y - sd.lam * lap.y - sd.gam * xc.y);
    gv = make_float2(gv.x + g1v.x - ad.x, gv.y + g1v.y - ad.y);
    oa.g[pp] = gv;
  }
  return gv;  // g after the step
}

// ------------------------------------------------------- TV shrink/update
// D_x x = x[i,j] - x[i-1,j], D_y x = x[i,j] - x[i,j-1] (periodic);
// v = D x + b;  d = shrink(v, 1/lam);  b <- v - d;  u = d - b (the next
// right-hand side uses D^H u).  With no wavelet the same is done on x itself
// with threshold 1/gam.
__global__ __launch_bounds__(256) void k_tv_shrink(Ws w, int only_nowavelet, int fresh, OuterArgs oa,
                                                   const float2* __restrict__ x, const float2* __restrict__ bxi,
                                                   const float2* __restrict__ byi,
                                                   float2* __restrict__ bx, float2* __restrict__ by,
                                                   float2* __restrict__ ux, float2* __restrict__ uy,
                                                   float2* __restrict__ bw, float2* __restrict__ uw) {
  if (oa.rec.counter && blockIdx.x == 0 && blockIdx.y == 0) record_solve(w, oa.rec);
  const int s = blockIdx.y;
  const SliceDev sd = w.sl[s];
  if (only_nowavelet && sd.levels > 0 && sd.wavelet != 0) return;
  const int m = sd.m, n = sd.n;
  const long long np = (long long)m * n;
  const float tl = 1.0f / sd.lam, tg = 1.0f / sd.gam;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < np; p += (long long)gridDim.x * blockDim.x) {
    const int i = int(p / n), j = int(p % n);
    const long long o = sd.img;
    const float2 xc = x[o + p];
    const float2 xu = x[o + (long long)((i - 1 + m) % m) * n + j];
    const float2 xl = x[o + (long long)i * n + (j - 1 + n) % n];
    if (oa.mode) {
      const float2 xd = x[o + (long long)((i + 1) % m) * n + j];
      const float2 xr = x[o + (long long)i * n + (j + 1) % n];
      const float2 lap = make_float2(4.f * xc.x - xu.x - xd.x - xl.x - xr.x, 4.f * xc.y - xu.y - xd.y - xl.y - xr.y);
      const float2 gv = oa.mode == 2 ? oa.g[o + p] : make_float2(0.f, 0.f);
      const float2 g1v = oa.mode == 2 ? oa.g1[o + p] : make_float2(0.f, 0.f);
      outer_at(sd, oa, o + p, xc, lap, oa.b[o + p], oa.r[o + p], gv, g1v);
    }
    const float2 zero = make_float2(0.f, 0.f);
    {
      const float2 v = cadd(csub(xc, xu), fresh ? zero : bxi[o + p]);
      const float2 d = shrink(v, tl);
      const float2 b = csub(v, d);
      bx[o + p] = b;
      ux[o + p] = csub(d, b);
    }
    {
      const float2 v = cadd(csub(xc, xl), fresh ? zero : byi[o + p]);
      const float2 d = shrink(v, tl);
      const float2 b = csub(v, d);
      by[o + p] = b;
      uy[o + p] = csub(d, b);
    }
    if (sd.levels == 0 || sd.wavelet == 0) {
      const float2 v = cadd(xc, fresh ? zero : bw[o + p]);
      const float2 d = shrink(v, tg);
      const float2 b = csub(v, d);
      bw[o + p] = b;
      uw[o + p] = csub(d, b);
    }
  }
}

// right-hand side g + lam (D_x^H u_x + D_y^H u_y) + gam * wv at pixel (i, j)
__device__ __forceinline__ float2 rhs_at(const SliceDev& sd, long long o, int i, int j, const float2* g,
                                         const float2* ux, const float2* uy, float2 wv) {
  const int m = sd.m, n = sd.n;
  const long long p = (long long)i * n + j;
  const float2 a = csub(ux[o + p], ux[o + (long long)((i + 1) % m) * n + j]);
  const float2 b = csub(uy[o + p], uy[o + (long long)i * n + (j + 1) % n]);
  const float2 gv = g[o + p];
  return make_float2(gv.x + sd.lam * (a.x + b.x) + sd.gam * wv.x, gv.y + sd.lam * (a.y + b.y) + sd.gam * wv.y);
}

__global__ __launch_bounds__(256) void k_rhs_nowavelet(Ws w, const float2* __restrict__ g,
                                                       const float2* __restrict__ ux, const float2* __restrict__ uy,
                                                       const float2* __restrict__ uw, float2* __restrict__ rhs) {
  const int s = blockIdx.y;
  const SliceDev sd = w.sl[s];
  if (sd.levels > 0 && sd.wavelet != 0) return;  // the wavelet synthesis writes these
  const long long np = (long long)sd.m * sd.n;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < np; p += (long long)gridDim.x * blockDim.x) {
    const int i = int(p / sd.n), j = int(p % sd.n);
    rhs[sd.img + p] = rhs_at(sd, sd.img, i, j, g, ux, uy, uw[sd.img + p]);
  }
}

// ---------------------------------------------------------------- wavelets
// Level l acts on the top-left (m >> l) x (n >> l) block (row stride n).
// Analysis, pass 0 (along axis 1):  tmp[i][k] = sum_t h[t] in[i][(2k+t) mod nl],
//                                   tmp[i][nl/2 + k] = sum_t g[t] in[...]
// Analysis, pass 1 (along axis 0):  coefficient rows k and ml/2 + k; the
// approximation block goes to `llout` unless this is the last level, every
// other coefficient is final and is either stored (`coef`) or consumed by the
// shrink/update of Algorithm 1 steps 8 and 11 (bw, uw).
// Synthesis is the transpose: pass 0 along axis 0, pass 1 along axis 1; the
// finest level's pass 1 can emit the right-hand side directly.


__device__ __forceinline__ int filt_len(int wavelet) { return wavelet == 1 ? 2 : 8; }
__device__ __forceinline__ float filt_h(int wavelet, int t) { return wavelet == 1 ? c_haar[t] : c_db4[t]; }
__device__ __forceinline__ float filt_g(int wavelet, int t) {
  const int K = filt_len(wavelet);
  const float v = filt_h(wavelet, K - 1 - t);
  return (t & 1) ? -v : v;
}

// bwv: a.bw[pos], loaded by the caller (shrink mode only)
__device__ __forceinline__ void coef_out(const SliceDev& sd, const WaveArgs& a, long long pos, float2 c, float2 bwv) {
  if (a.mode == 0) {
    a.coef[pos] = c;
  } else {
    const float2 v = cadd(c, bwv);
    const float2 d = shrink(v, 1.0f / sd.gam);
    const float2 b = csub(v, d);
    a.bw[pos] = b;
    a.uw[pos] = csub(d, b);
  }
}

// Both passes of one level in a workgroup: an output tile of kWT x kWT
// coefficients in each of the four bands, from an input tile of
// (2 kWT + 7)^2 pixels (filter support plus, at level 0, the row above and the
// column to the left for the fused TV step), all with periodic wrap.
constexpr int kWT = 16;
constexpr int kWIn = 2 * kWT + 7;  // 39: 1 TV halo + 2 kWT + 6 filter halo
constexpr int kWThreads = 256;     // workgroup size of both wavelet kernels

template <int K>
struct Filt {
  float h[K], g[K];
  __device__ __forceinline__ Filt() {
#pragma unroll
    for (int t = 0; t < K; ++t) {
      h[t] = K == 2 ? c_haar[t] : c_db4[t];
      const float v = K == 2 ? c_haar[K - 1 - t] : c_db4[K - 1 - t];
      g[t] = (t & 1) ? -v : v;
    }
  }
};

// index i in [-L, 2L) folded into [0, L); any i when `small`
__device__ __forceinline__ int wrap(int i, int L, bool small) {
  if (small) return ((i % L) + L) % L;
  return i < 0 ? i + L : (i >= L ? i - L : i);
}

template <int K>
__device__ __forceinline__ void dwt_ana_tile(const SliceDev& sd, const WaveArgs& a, const TvArgs& tv,
                                             float2 (*tile)[kWIn + 1], float2 (*rowb)[2 * kWT + 1],
                                             float2 (*uys)[2 * kWT + 1], int bt) {
  const int n = sd.n;
  const int ml = sd.m >> a.level, nl = n >> a.level;
  const int mh = ml / 2, nh = nl / 2;
  const int tcols = (nh + kWT - 1) / kWT;
  const int k0 = (bt / tcols) * kWT, c0 = (bt % tcols) * kWT;
  const long long o = sd.img;
  const bool lastlev = (a.level == sd.levels - 1);
  const bool small = ml < kWIn || nl < kWIn;
  const Filt<K> f;
  // Every operand the kernel will need besides the input tile is requested
  // first, so that it is in flight during the tile load and both passes:
  // the Bregman variables of the outputs (shrink mode) and, at level 0, the
  // TV and outer-update operands of the 2 kWT x 2 kWT pixel block.
  constexpr int PER = kWT * 2 * kWT / kWThreads;
  float2 blo[PER] = {}, bhi[PER] = {};
  if (a.mode == 1 && !a.fresh) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = threadIdx.x + kWThreads * e;
      const int k = idx / (2 * kWT), cp = idx % (2 * kWT);
      const int half = cp / kWT, gk = k0 + k, gc = c0 + (cp % kWT);
      if (gk < mh && gc < nh) {
        const long long plo = o + (long long)gk * n + half * nh + gc;
        const long long phi = o + (long long)(mh + gk) * n + half * nh + gc;
        if (!(half == 0 && !lastlev)) blo[e] = a.bw[plo];
        bhi[e] = a.bw[phi];
      }
    }
  }
  // Level 0 covers whole 2 kWT x 2 kWT pixel blocks (image sides are
  // multiples of 32); the TV step also needs b_x on the row below the block
  // and b_y on the column to its right (threads 0 .. 4 kWT - 1, one each).
  constexpr int PER_TV = 4 * kWT * kWT / kWThreads;
  const OuterArgs& oa = tv.outer;
  const bool tv_here = tv.enabled && a.level == 0;
  float2 bxs[PER_TV] = {}, bys[PER_TV] = {}, obs[PER_TV], ors[PER_TV], ogs[PER_TV] = {}, og1s[PER_TV] = {};
  float2 bhalo = make_float2(0.f, 0.f);
  if (tv_here) {
#pragma unroll
    for (int e = 0; e < PER_TV; ++e) {
      const int idx = threadIdx.x + kWThreads * e;
      const int ia = idx / (2 * kWT), jb = idx % (2 * kWT);
      const long long pp = o + (long long)(2 * k0 + ia) * n + 2 * c0 + jb;
      if (!tv.fresh) {
        bxs[e] = tv.bxi[pp];
        bys[e] = tv.byi[pp];
      }
      ogs[e] = oa.g[pp];
      if (oa.mode) {
        obs[e] = oa.b[pp];
        ors[e] = oa.r[pp];
        if (oa.mode == 2) og1s[e] = oa.g1[pp];
      }
    }
    if (!tv.fresh && threadIdx.x < 4 * kWT) {
      const int t = threadIdx.x;
      const int id = (2 * k0 + 2 * kWT) % ml, jr = (2 * c0 + 2 * kWT) % nl;
      bhalo = t < 2 * kWT ? tv.bxi[o + (long long)id * n + 2 * c0 + t]
                          : tv.byi[o + (long long)(2 * k0 + t - 2 * kWT) * n + jr];
    }
  }
  {
    // every load of the thread in flight at once, then the LDS stores
    constexpr int PER = (kWIn * kWIn + kWThreads - 1) / kWThreads;
    float2 v[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = threadIdx.x + kWThreads * e;
      if (idx < kWIn * kWIn) {
        const int ra = idx / kWIn, cb = idx % kWIn;
        const int r = wrap(2 * k0 - 1 + ra, ml, small), c = wrap(2 * c0 - 1 + cb, nl, small);
        v[e] = a.in[o + (long long)r * n + c];
      }
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = threadIdx.x + kWThreads * e;
      if (idx < kWIn * kWIn) tile[idx / kWIn][idx % kWIn] = v[e];
    }
  }
  __syncthreads();
  // along axis 1
  for (int idx = threadIdx.x; idx < (kWIn - 1) * kWT; idx += blockDim.x) {
    const int ra = 1 + idx / kWT, c = idx % kWT;
    float2 lo = make_float2(0.f, 0.f), hi = make_float2(0.f, 0.f);
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const float2 v = tile[ra][1 + 2 * c + t];
      lo = make_float2(lo.x + f.h[t] * v.x, lo.y + f.h[t] * v.y);
      hi = make_float2(hi.x + f.g[t] * v.x, hi.y + f.g[t] * v.y);
    }
    rowb[ra][c] = lo;
    rowb[ra][kWT + c] = hi;
  }
  __syncthreads();
  // along axis 0, then the band placement (Mallat layout)
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int idx = threadIdx.x + kWThreads * e;
    const int k = idx / (2 * kWT), cp = idx % (2 * kWT);
    const int half = cp / kWT, gk = k0 + k, gc = c0 + (cp % kWT);
    if (gk >= mh || gc >= nh) continue;
    float2 lo = make_float2(0.f, 0.f), hi = make_float2(0.f, 0.f);
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const float2 v = rowb[1 + 2 * k + t][cp];
      lo = make_float2(lo.x + f.h[t] * v.x, lo.y + f.h[t] * v.y);
      hi = make_float2(hi.x + f.g[t] * v.x, hi.y + f.g[t] * v.y);
    }
    const long long plo = o + (long long)gk * n + half * nh + gc;
    const long long phi = o + (long long)(mh + gk) * n + half * nh + gc;
    if (half == 0 && !lastlev) a.out[plo] = lo;  // approximation block feeds the next level
    else coef_out(sd, a, plo, lo, blo[e]);
    coef_out(sd, a, phi, hi, bhi[e]);
  }
  // level 0: Algorithm 1 steps 6, 7, 9, 10 on the 2 kWT x 2 kWT pixel block,
  // the outer update (steps 13-15), and the TV part of the next right-hand
  // side (step 4): tvr = g + lam (D_x^H u_x + D_y^H u_y), with u_x on the row
  // below the block and u_y on the column to its right recomputed here
  if (tv_here) {
    __syncthreads();  // rowb is reused for u_x once the axis-0 pass has read it
    float2 (*uxs)[2 * kWT + 1] = rowb;
    const float thr = 1.0f / sd.lam;
    float2 gs[PER_TV];
#pragma unroll
    for (int e = 0; e < PER_TV; ++e) {
      const int idx = threadIdx.x + kWThreads * e;
      const int ia = idx / (2 * kWT), jb = idx % (2 * kWT);
      const long long pp = o + (long long)(2 * k0 + ia) * n + 2 * c0 + jb;
      const float2 xc = tile[1 + ia][1 + jb], xu = tile[ia][1 + jb], xl = tile[1 + ia][jb];
      gs[e] = ogs[e];
      if (oa.mode) {
        const float2 xd = tile[2 + ia][1 + jb], xr = tile[1 + ia][2 + jb];
        const float2 lap = make_float2(4.f * xc.x - xu.x - xd.x - xl.x - xr.x, 4.f * xc.y - xu.y - xd.y - xl.y - xr.y);
        gs[e] = outer_at(sd, oa, pp, xc, lap, obs[e], ors[e], ogs[e], og1s[e]);
      }
      {
        const float2 v = cadd(csub(xc, xu), bxs[e]);
        const float2 d = shrink(v, thr);
        const float2 b = csub(v, d);
        tv.bx[pp] = b;
        uxs[ia][jb] = csub(d, b);
      }
      {
        const float2 v = cadd(csub(xc, xl), bys[e]);
        const float2 d = shrink(v, thr);
        const float2 b = csub(v, d);
        tv.by[pp] = b;
        uys[ia][jb] = csub(d, b);
      }
    }
    if (threadIdx.x < 4 * kWT) {
      const int t = threadIdx.x;
      if (t < 2 * kWT) {  // u_x on the row below the block
        const float2 v = cadd(csub(tile[1 + 2 * kWT][1 + t], tile[2 * kWT][1 + t]), bhalo);
        const float2 d = shrink(v, thr);
        uxs[2 * kWT][t] = csub(d, csub(v, d));
      } else {  // u_y on the column to the right
        const int ia = t - 2 * kWT;
        const float2 v = cadd(csub(tile[1 + ia][1 + 2 * kWT], tile[1 + ia][2 * kWT]), bhalo);
        const float2 d = shrink(v, thr);
        uys[ia][2 * kWT] = csub(d, csub(v, d));
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PER_TV; ++e) {
      const int idx = threadIdx.x + kWThreads * e;
      const int ia = idx / (2 * kWT), jb = idx % (2 * kWT);
      const long long pp = o + (long long)(2 * k0 + ia) * n + 2 * c0 + jb;
      const float2 x0 = uxs[ia][jb], x1 = uxs[ia + 1][jb], y0 = uys[ia][jb], y1 = uys[ia][jb + 1];
      tv.tvr[pp] = make_float2(gs[e].x + sd.lam * ((x0.x - x1.x) + (y0.x - y1.x)),
                               gs[e].y + sd.lam * ((x0.y - x1.y) + (y0.y - y1.y)));
    }
  }
}

__global__ __launch_bounds__(256) void k_dwt_ana(Ws w, WaveArgs a, TvArgs tv) {
  __shared__ float2 tile[kWIn][kWIn + 1];
  __shared__ float2 rowb[kWIn][2 * kWT + 1];
  __shared__ float2 uys[2 * kWT][2 * kWT + 1];
  if (tv.outer.rec.counter && blockIdx.x == 0 && blockIdx.y == 0) record_solve(w, tv.outer.rec);
  const SliceDev sd = w.sl[blockIdx.y];
  if (sd.wavelet == 0 || a.level >= sd.levels) return;
  const int mh = (sd.m >> a.level) / 2, nh = (sd.n >> a.level) / 2;
  const int bt = xcd_tile(blockIdx.x, gridDim.x);
  if (bt >= ((nh + kWT - 1) / kWT) * ((mh + kWT - 1) / kWT)) return;
  if (sd.wavelet == 1) dwt_ana_tile<2>(sd, a, tv, tile, rowb, uys, bt);
  else dwt_ana_tile<8>(sd, a, tv, tile, rowb, uys, bt);
}

// Synthesis of one level: a 2 kWT x 2 kWT output pixel block from the four
// bands' (kWT + 3)^2 coefficient windows; at level 0 in mode 1 the pixel is
// combined straight into the Split Bregman right-hand side.  Output rows (and
// columns) 2a and 2a + 1 read the same coefficients, with the even and the
// odd filter taps, so each work item produces such a pair.
constexpr int kWB = kWT + 3;

template <int K>
__device__ __forceinline__ void dwt_syn_tile(const SliceDev& sd, const WaveArgs& a, float2 (*bands)[kWB][kWB + 1],
                                             float2 (*u)[2 * kWB + 1], int bt) {
  const int n = sd.n;
  const int ml = sd.m >> a.level, nl = n >> a.level;
  const int mh = ml / 2, nh = nl / 2;
  const int tcols = (nh + kWT - 1) / kWT;
  const int k0 = (bt / tcols) * kWT, c0 = (bt % tcols) * kWT;
  const long long o = sd.img;
  const bool lastlev = (a.level == sd.levels - 1);
  const bool small = mh < kWB || nh < kWB;
  const Filt<K> f;
  // pixel pairs (columns 2b, 2b + 1 of the block) per thread in the last pass
  constexpr int PP = 2 * kWT * kWT / kWThreads;
  // the right-hand side's TV part (level 0, mode 1) is requested first so
  // that it is in flight during the band loads and both filter passes; the
  // workspace images are 16-byte aligned
  const bool rhs_mode = a.level == 0 && a.mode == 1;
  float4 rt[PP];
  if (rhs_mode) {
#pragma unroll
    for (int e = 0; e < PP; ++e) {
      const int pidx = threadIdx.x + kWThreads * e;
      const int ia = pidx / kWT, b = pidx % kWT;
      const int i = 2 * k0 + ia, jj = 2 * c0 + 2 * b;
      if (i < ml && jj < nl) rt[e] = *reinterpret_cast<const float4*>(a.tvr + o + (long long)i * n + jj);
    }
  }
  {
    constexpr int NB = 4 * kWB * kWB;
    constexpr int PER = (NB + kWThreads - 1) / kWThreads;
    float2 v[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = threadIdx.x + kWThreads * e;
      if (idx < NB) {
        const int b = idx / (kWB * kWB), rr = (idx / kWB) % kWB, cc = idx % kWB;
        const int a0 = b >> 1, a1 = b & 1;
        const int kr = wrap(k0 - 3 + rr, mh, small), kc = wrap(c0 - 3 + cc, nh, small);
        const float2* src = (a0 == 0 && a1 == 0 && !lastlev) ? a.in : a.coef;
        v[e] = src[o + (long long)(a0 * mh + kr) * n + a1 * nh + kc];
      }
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = threadIdx.x + kWThreads * e;
      if (idx < NB) bands[idx / (kWB * kWB)][(idx / kWB) % kWB][idx % kWB] = v[e];
    }
  }
  __syncthreads();
  // along axis 0: rows 2 r and 2 r + 1 of u from band rows r - t + 3
  for (int idx = threadIdx.x; idx < kWT * 2 * kWB; idx += blockDim.x) {
    const int r = idx / (2 * kWB), q = idx % (2 * kWB);
    const int a1 = q / kWB, cc = q % kWB;
    float2 ev = make_float2(0.f, 0.f), od = make_float2(0.f, 0.f);
#pragma unroll
    for (int tt = 0; tt < K / 2; ++tt) {
      const float2 lv = bands[a1][r - tt + 3][cc], hv = bands[2 + a1][r - tt + 3][cc];
      ev = make_float2(ev.x + f.h[2 * tt] * lv.x + f.g[2 * tt] * hv.x,
                       ev.y + f.h[2 * tt] * lv.y + f.g[2 * tt] * hv.y);
      od = make_float2(od.x + f.h[2 * tt + 1] * lv.x + f.g[2 * tt + 1] * hv.x,
                       od.y + f.h[2 * tt + 1] * lv.y + f.g[2 * tt + 1] * hv.y);
    }
    u[2 * r][q] = ev;
    u[2 * r + 1][q] = od;
  }
  __syncthreads();
  // along axis 1: pixel columns 2 b and 2 b + 1 from u columns b - t + 3
#pragma unroll
  for (int e = 0; e < PP; ++e) {
    const int pidx = threadIdx.x + kWThreads * e;
    const int ia = pidx / kWT, b = pidx % kWT;
    const int i = 2 * k0 + ia, jj = 2 * c0 + 2 * b;
    if (i >= ml || jj >= nl) continue;
    float2 ev = make_float2(0.f, 0.f), od = make_float2(0.f, 0.f);
#pragma unroll
    for (int tt = 0; tt < K / 2; ++tt) {
      const float2 lv = u[ia][b - tt + 3], hv = u[ia][kWB + b - tt + 3];
      ev = make_float2(ev.x + f.h[2 * tt] * lv.x + f.g[2 * tt] * hv.x,
                       ev.y + f.h[2 * tt] * lv.y + f.g[2 * tt] * hv.y);
      od = make_float2(od.x + f.h[2 * tt + 1] * lv.x + f.g[2 * tt + 1] * hv.x,
                       od.y + f.h[2 * tt + 1] * lv.y + f.g[2 * tt + 1] * hv.y);
    }
    const long long p = o + (long long)i * n + jj;
    if (rhs_mode) {
      // Algorithm 1 step 4: [g + lam (D_x^H u_x + D_y^H u_y)] + gam W^H u_w
      const float gam = sd.gam;
      const float4 t = rt[e];
      *reinterpret_cast<float4*>(a.rhs + p) =
          make_float4(t.x + gam * ev.x, t.y + gam * ev.y, t.z + gam * od.x, t.w + gam * od.y);
    } else {
      a.out[p] = ev;
      a.out[p + 1] = od;
    }
  }
}

__global__ __launch_bounds__(256) void k_dwt_syn(Ws w, WaveArgs a) {
  __shared__ float2 bands[4][kWB][kWB + 1];
  __shared__ float2 u[2 * kWT][2 * kWB + 1];
  const SliceDev sd = w.sl[blockIdx.y];
  if (sd.wavelet == 0 || a.level >= sd.levels) return;
  const int mh = (sd.m >> a.level) / 2, nh = (sd.n >> a.level) / 2;
  const int bt = xcd_tile(blockIdx.x, gridDim.x);
  if (bt >= ((nh + kWT - 1) / kWT) * ((mh + kWT - 1) / kWT)) return;
  if (sd.wavelet == 1) dwt_syn_tile<2>(sd, a, bands, u, bt);
  else dwt_syn_tile<8>(sd, a, bands, u, bt);
}

// ------------------------------------------------------ spectrum assembly
// k(u, v) = mu k_c(u) + lam (4 - 2 cos(2 pi u / m) - 2 cos(2 pi v / n)) + gam
// for a line mask, k_c(u) = (1/N^2) sum_l r(l) Pbar(l - u); optional
// multiplicative correction; outputs k, 1 / (k m n) and the Jacobi inverse
// diagonal 1 / (mu |Omega|/N sum_c |S_c|^2 + 4 lam + gam).
// One workgroup per slice: k_c along the lines and the row part of k,
//   krow(u) = mu k_c(u) + lam (2 - 2 cos(2 pi u / m)) + gam,
// and the sampled fraction |Omega| / m, written over the slice's Pbar
// partials (krow at [0, m), the fraction at m) once they are summed.
__global__ __launch_bounds__(256) void k_build_krow(Ws w, double* __restrict__ pbar) {
  __shared__ double sp[1024];
  __shared__ int smk[1024];
  __shared__ int ssum;
  const int s = blockIdx.x;
  const SliceDev sd = w.sl[s];
  if (sd.mask_kind != 0) return;  // 2D masks: k_build_k2d
  const int m = sd.m, n = sd.n;
  const int ntile = n / col_tile(m);
  const uint8_t* mk = w.mask + sd.mask;
  double* pb = pbar + sd.aux;
  if (threadIdx.x == 0) ssum = 0;
  __syncthreads();
  int cnt = 0;
  for (int u = threadIdx.x; u < m; u += blockDim.x) {
    double a = 0.0;
#pragma unroll 16
    for (int tl = 0; tl < ntile; ++tl) a += pb[(long long)tl * m + u];
    sp[u] = a * n;
    smk[u] = mk[u] ? 1 : 0;
    cnt += mk[u] ? 1 : 0;
  }
  atomicAdd(&ssum, cnt);
  __syncthreads();
  const double N = (double)m * n;
  for (int u = threadIdx.x; u < m; u += blockDim.x) {
    double a = 0.0;
#pragma unroll 16
    for (int l = 0; l < m; ++l) {
      const int d = l - u;
      const double pv = sp[d < 0 ? d + m : d];
      if (smk[l]) a += pv;
    }
    pb[u] = (double)sd.mu * (a / (N * N)) + (double)sd.lam * (2.0 - 2.0 * cospi(2.0 * u / m)) + (double)sd.gam;
  }
  if (threadIdx.x == 0) pb[m] = (double)ssum / m;
}

// k(u, v) = krow(u) + lam (2 - 2 cos(2 pi v / n)), a row band per workgroup.
__global__ __launch_bounds__(256) void k_build_k(Ws w, const double* __restrict__ pbar, const float* __restrict__ corr,
                                                 float* __restrict__ kraw, float* __restrict__ kinv,
                                                 float* __restrict__ jac, int* __restrict__ bad) {
  __shared__ double sdv[1024];
  const int s = blockIdx.y;
  const SliceDev sd = w.sl[s];
  if (sd.mask_kind != 0) return;
  const int m = sd.m, n = sd.n;
  const double* pb = pbar + sd.aux;
  const int u0 = (int)((long long)blockIdx.x * m / gridDim.x), u1 = (int)((long long)(blockIdx.x + 1) * m / gridDim.x);
  for (int v = threadIdx.x; v < n; v += blockDim.x) sdv[v] = (double)sd.lam * (2.0 - 2.0 * cospi(2.0 * v / n));
  __syncthreads();
  const double N = (double)m * n;
  const double frac = pb[m];
  const long long np = (long long)(u1 - u0) * n;
  int badl = 0;
  for (long long q = threadIdx.x; q < np; q += blockDim.x) {
    const int du = int(q / n), v = int(q - (long long)du * n);
    const long long p = (long long)(u0 + du) * n + v;
    double k = pb[u0 + du] + sdv[v];
    if (corr) k *= (double)corr[sd.img + p];
    if (!(k > 0.0) || !isfinite(k)) badl = 1;
    kraw[sd.img + p] = (float)k;
    kinv[sd.img + p] = (float)(1.0 / (k * N));
    const double dA = (double)sd.mu * frac * (double)jac[sd.img + p] + 4.0 * sd.lam + sd.gam;
    jac[sd.img + p] = (float)(1.0 / dA);
  }
  if (badl) atomicOr(bad, 1);
}

// y += gam W^H W x, given wx = W^H W x (x itself for slices without a wavelet)
__global__ __launch_bounds__(256) void k_add_gamma(Ws w, const float2* __restrict__ wx, const float2* __restrict__ x,
                                                   float2* __restrict__ y) {
  const int s = blockIdx.y;
  const SliceDev sd = w.sl[s];
  const long long np = (long long)sd.m * sd.n;
  const float2* src = (sd.levels > 0 && sd.wavelet != 0) ? wx : x;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < np; p += (long long)gridDim.x * blockDim.x) {
    const float2 a = src[sd.img + p], b = y[sd.img + p];
    y[sd.img + p] = make_float2(b.x + sd.gam * a.x, b.y + sd.gam * a.y);
  }
}

__global__ void k_fill(float2* p, long long count, float2 v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

// ============================================================== launchers

static dim3 simple_grid(const Simple& S) {
  long long blocks = (S.max_pixels + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  return dim3((unsigned)blocks, S.nslices);
}

hipError_t launch_pcg_check(hipStream_t st, const Ws& w, int nslices, double tol, int setup, float2* x) {
  hipLaunchKernelGGL(k_pcg_check, dim3(nslices), dim3(256), 0, st, w, tol, setup, x);
  return hipGetLastError();
}

hipError_t launch_set_int(hipStream_t st, int* p, int v) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, p, v);
  return hipGetLastError();
}

hipError_t launch_tv_shrink(const Simple& S, const Ws& w, int only_nowavelet, int fresh, const OuterArgs& oa,
                            const float2* x, const float2* bxi, const float2* byi, float2* bx, float2* by, float2* ux,
                            float2* uy, float2* bw, float2* uw) {
  hipLaunchKernelGGL(k_tv_shrink, simple_grid(S), dim3(256), 0, S.stream, w, only_nowavelet, fresh, oa, x, bxi, byi,
                     bx, by, ux, uy, bw, uw);
  return hipGetLastError();
}

hipError_t launch_rhs_nowavelet(const Simple& S, const Ws& w, const float2* g, const float2* ux, const float2* uy,
                                const float2* uw, float2* rhs) {
  hipLaunchKernelGGL(k_rhs_nowavelet, simple_grid(S), dim3(256), 0, S.stream, w, g, ux, uy, uw, rhs);
  return hipGetLastError();
}

int wavelet_tiles(int m, int n, int level) {
  const int mh = (m >> level) / 2, nh = (n >> level) / 2;
  return ((mh + kWT - 1) / kWT) * ((nh + kWT - 1) / kWT);
}

hipError_t launch_wavelet(const Simple& S, const Ws& w, const WaveArgs& a, const TvArgs& tv, int tiles) {
  const dim3 grid((unsigned)std::max(1, tiles), S.nslices);
  if (a.inverse)
    hipLaunchKernelGGL(k_dwt_syn, grid, dim3(256), 0, S.stream, w, a);
  else
    hipLaunchKernelGGL(k_dwt_ana, grid, dim3(256), 0, S.stream, w, a, tv);
  return hipGetLastError();
}

hipError_t launch_build_k(const Simple& S, const Ws& w, double* pbar, const float* corr, float* kraw,
                          float* kinv, float* jac, int* bad) {
  hipLaunchKernelGGL(k_build_krow, dim3(S.nslices), dim3(256), 0, S.stream, w, pbar);
  dim3 grid = simple_grid(S);
  if (grid.x > 64) grid.x = 64;
  hipLaunchKernelGGL(k_build_k, grid, dim3(256), 0, S.stream, w, pbar, corr, kraw, kinv, jac, bad);
  return hipGetLastError();
}

hipError_t launch_add_gamma(const Simple& S, const Ws& w, const float2* wx, const float2* x, float2* y) {
  hipLaunchKernelGGL(k_add_gamma, simple_grid(S), dim3(256), 0, S.stream, w, wx, x, y);
  return hipGetLastError();
}

hipError_t launch_fill(hipStream_t st, float2* p, long long count, float2 v) {
  long long blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, p, count, v);
  return hipGetLastError();
}

}  // namespace pics

// System operator and spectrum build for fully random 2D sampling masks
// (Methods, Undersampling: the second scheme).  A 2D mask does not factor
// along one axis, so each coil needs a full 2D transform pair; the operator
// runs as three passes through a coil-image buffer ([nc][m][n] per slice):
//   1. row tiles:    u_c = row-FFT(S_c p)                       (all coils)
//   2. column tiles: u_c = col-IFFT(r / N . col-FFT(u_c))        (all coils)
//   3. row tiles:    q = mu sum_c conj(S_c) row-IFFT(u_c)
//                        + lam (D_x^H D_x + D_y^H D_y) p + gam p
// (Eq. system with W^H W = I).  In the PCG mode pass 1 also forms
// p = z + beta p_old and pass 3 the sigma = Re(p^H A p) partials, as the
// line-mask kernel does.
//
// The circulant spectrum of a 2D mask is the full 2D cross-correlation
// k_c(j) = (1/N^2) sum_l r(l) P(l - j), P = sum_c |DFT(s_c)|^2 (Eqs. d,
// diagonalelements), evaluated with FFTs: k_c = IDFT(DFT(r) conj(DFT(P))) / N^3
// for the unnormalised transforms used here.
#include "tiles.hpp"

namespace pics {

// ------------------------------------------------------------------ pass 1
template <int N, int MODE>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void k_row_sp(Ws w, int pk, double tol, const float2* __restrict__ xin,
                                                               const float2* __restrict__ zsrc,
                                                               const float2* __restrict__ pold, float2* __restrict__ pn,
                                                               float2* __restrict__ coil) {
  constexpr int NT = RowCfg<N>::NT, E = RowCfg<N>::E, TH = RowCfg<N>::THREADS;
  __shared__ float2 lds[RowCfg<N>::LDS];
  __shared__ float2 s_tw[N];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  const int t = threadIdx.x % NT, rr_ = threadIdx.x / NT;
  const int i = blockIdx.x * kRowRR + rr_;
  const long long row = sd.img + (long long)i * N;

  float beta = 0.f;
  bool first = true;
  if (MODE == CA_PCG) {
    const PcgState* st = w.st + s;
    if (st->done) return;
    int status;
    if (pcg_should_stop(w, s, sd.m, tol, &status)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) pcg_mark_done(w, s, status, tol);
      return;
    }
    const int it = st->it_a;
    first = (it == 0);
    if (!first) {
      const int nrt = sd.m / kRowRR;
      const double rho_i = part_sum(part_ptr(w.part, s, P_RHO0 + (it & 1)), nrt);
      const double rho_p = part_sum(part_ptr(w.part, s, P_RHO0 + ((it - 1) & 1)), nrt);
      beta = float(rho_i / rho_p);
    }
  }
  stage_twiddles<N, TH>(s_tw, w.tw);

  float2 pv[E];
  if (MODE != CA_PCG) {
#pragma unroll
    for (int e = 0; e < E; ++e) pv[e] = xin[row + t + NT * e];
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) pv[e] = zsrc[row + t + NT * e];
    if (pk == PK_JACOBI) {
#pragma unroll
      for (int e = 0; e < E; ++e) pv[e] = cscale(pv[e], w.jac[row + t + NT * e]);
    }
    if (!first) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const float2 o = pold[row + t + NT * e];
        pv[e] = make_float2(pv[e].x + beta * o.x, pv[e].y + beta * o.y);
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) pn[row + t + NT * e] = pv[e];
  }
  // the next coil's maps are loaded while this coil is transformed (not at
  // length 1024: 1024-thread workgroups leave no registers for them)
  const long long plane = (long long)sd.m * N;
  const long long row0 = sd.coil + (long long)i * N + t;
  if constexpr (N < 1024) {
    float2 sv[E], sn[E];
#pragma unroll
    for (int e = 0; e < E; ++e) sv[e] = w.sens[row0 + NT * e];
    for (int c = 0; c < sd.nc; ++c) {
      const long long crow = row0 + c * plane;
      {
        // unconditional (the last trip reloads its own maps): a conditional
        // load makes the compiler wait on it before the transform
        const long long nx = c + 1 < sd.nc ? plane : 0;
#pragma unroll
        for (int e = 0; e < E; ++e) sn[e] = w.sens[crow + nx + NT * e];
      }
      float2 v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = cmul(sv[e], pv[e]);
      fft<N, -1, RowLay<N>>(v, t, lds, rr_, s_tw);
#pragma unroll
      for (int e = 0; e < E; ++e) coil[crow + NT * e] = v[e];
#pragma unroll
      for (int e = 0; e < E; ++e) sv[e] = sn[e];
    }
  } else {
    for (int c = 0; c < sd.nc; ++c) {
      const long long crow = row0 + c * plane;
      float2 v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = cmul(w.sens[crow + NT * e], pv[e]);
      fft<N, -1, RowLay<N>>(v, t, lds, rr_, s_tw);
#pragma unroll
      for (int e = 0; e < E; ++e) coil[crow + NT * e] = v[e];
    }
  }
}

// ------------------------------------------------------------------ pass 2
// use_state: skip slices whose PCG solve has finished.
template <int M>
__global__ __launch_bounds__(ColCfg<M>::THREADS) void k_col_mask2d(Ws w, int use_state, float2* __restrict__ coil) {
  constexpr int NT = ColCfg<M>::NT, E = ColCfg<M>::E, T = ColCfg<M>::T;
  __shared__ float2 lds[ColLay<T>::template size<M>];
  __shared__ float2 s_tw[M];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  if (use_state && w.st[s].done) return;
  const int n = sd.n;
  const int j = threadIdx.x % T, t = threadIdx.x / T;
  const int col = blockIdx.x * T + j;
  stage_twiddles<M, ColCfg<M>::THREADS>(s_tw, w.tw);
  const uint8_t* mk = w.mask + sd.mask;
  const float inv_n = 1.0f / ((float)M * (float)n);
  float sc[E];  // r(u, col) / N: the unitary pair's scale folded into the mask
#pragma unroll
  for (int e = 0; e < E; ++e) sc[e] = mk[(long long)(t + NT * e) * n + col] ? inv_n : 0.f;
  // the next coil's column is loaded while this coil is transformed
  const long long plane = (long long)M * n;
  float2 v[E], vn[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = coil[sd.coil + col + (long long)(t + NT * e) * n];
  for (int c = 0; c < sd.nc; ++c) {
    float2* cb = coil + sd.coil + c * plane + col;
    if (c > 0) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = vn[e];
    }
    {
      // unconditional (the last trip reloads its own column before writing
      // it; the copy is not used)
      const long long nx = c + 1 < sd.nc ? plane : 0;
#pragma unroll
      for (int e = 0; e < E; ++e) vn[e] = cb[nx + (long long)(t + NT * e) * n];
    }
    fft<M, -1, ColLay<T>>(v, t, lds, j, s_tw);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cscale(v[e], sc[e]);
    fft<M, +1, ColLay<T>>(v, t, lds, j, s_tw);
#pragma unroll
    for (int e = 0; e < E; ++e) cb[(long long)(t + NT * e) * n] = v[e];
  }
}

// ------------------------------------------------------------------ pass 3
template <int N>
struct Acc2dCfg {
  static constexpr int TILE = (kRowRR + 2) * N;  // p rows i0 - 1 .. i0 + RR
  static constexpr int LDS = RowCfg<N>::LDS > TILE ? RowCfg<N>::LDS : TILE;
};

template <int N, int MODE>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void k_row_acc(Ws w, int terms, const float2* __restrict__ xin,
                                                                const float2* __restrict__ pn,
                                                                const float2* __restrict__ coil,
                                                                float2* __restrict__ out) {
  constexpr int NT = RowCfg<N>::NT, E = RowCfg<N>::E, TH = RowCfg<N>::THREADS;
  __shared__ float2 lds[Acc2dCfg<N>::LDS];
  __shared__ float2 s_tw[N];
  __shared__ double red[16];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  const int m = sd.m;
  const int t = threadIdx.x % NT, rr_ = threadIdx.x / NT;
  const int i0 = blockIdx.x * kRowRR, i = i0 + rr_;
  const long long row = sd.img + (long long)i * N;
  int it = 0;
  if (MODE == CA_PCG) {
    const PcgState* st = w.st + s;
    if (st->done) return;
    it = st->it_a;
  }
  const float2* __restrict__ p = (MODE == CA_PCG ? pn : xin) + sd.img;
  stage_twiddles<N, TH>(s_tw, w.tw);

  float2 acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = make_float2(0.f, 0.f);
  if (terms & TERM_DATA) {
    // the coil's maps are requested with its row, the next coil's row and
    // maps while it is transformed (not at length 1024: no registers left)
    const long long plane = (long long)m * N;
    const long long row0 = sd.coil + (long long)i * N + t;
    if constexpr (N < 1024) {
      float2 v[E], sv[E], vn[E], sn[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        v[e] = coil[row0 + NT * e];
        sv[e] = w.sens[row0 + NT * e];
      }
      for (int c = 0; c < sd.nc; ++c) {
        const long long crow = row0 + c * plane;
        {
          // unconditional (the last trip reloads its own row and maps)
          const long long nx = c + 1 < sd.nc ? plane : 0;
#pragma unroll
          for (int e = 0; e < E; ++e) {
            vn[e] = coil[crow + nx + NT * e];
            sn[e] = w.sens[crow + nx + NT * e];
          }
        }
        fft<N, +1, RowLay<N>>(v, t, lds, rr_, s_tw);
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = cadd(acc[e], cconjmul(sv[e], v[e]));
#pragma unroll
        for (int e = 0; e < E; ++e) {
          v[e] = vn[e];
          sv[e] = sn[e];
        }
      }
    } else {
      for (int c = 0; c < sd.nc; ++c) {
        const long long crow = row0 + c * plane;
        float2 v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = coil[crow + NT * e];
        fft<N, +1, RowLay<N>>(v, t, lds, rr_, s_tw);
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = cadd(acc[e], cconjmul(w.sens[crow + NT * e], v[e]));
      }
    }
    __syncthreads();  // the transforms are done with the LDS buffer
  }
  // p rows i0 - 1 .. i0 + RR (periodic) for the Laplacian
  for (int k = threadIdx.x; k < (kRowRR + 2) * N; k += TH) {
    const int rr = k / N, col = k % N;
    const int gi = (i0 - 1 + rr + m) % m;
    lds[k] = p[(long long)gi * N + col];
  }
  __syncthreads();
  const float mu = sd.mu, lam = sd.lam, gam = sd.gam;
  double sig = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int col = t + NT * e;
    const float2 c0 = lds[(rr_ + 1) * N + col];
    float2 a = make_float2(mu * acc[e].x, mu * acc[e].y);
    if (terms & TERM_TV) {
      const float2 u = lds[rr_ * N + col], d = lds[(rr_ + 2) * N + col];
      const float2 l = lds[(rr_ + 1) * N + (col - 1 + N) % N], r = lds[(rr_ + 1) * N + (col + 1) % N];
      a = make_float2(a.x + lam * (4.f * c0.x - u.x - d.x - l.x - r.x), a.y + lam * (4.f * c0.y - u.y - d.y - l.y - r.y));
    }
    if (terms & TERM_GAMMA) a = make_float2(a.x + gam * c0.x, a.y + gam * c0.y);
    out[row + col] = a;
    sig += (double)c0.x * (double)a.x + (double)c0.y * (double)a.y;
  }
  if (MODE == CA_PCG) {
    sig = block_sum_f64(sig, red);
    if (threadIdx.x == 0) {
      part_ptr(w.part, s, P_SIGMA)[blockIdx.x] = sig;  // one partial per row tile
      if (blockIdx.x == 0) w.st[s].it_r = it;
    }
  }
}

// -------------------------------------------------------- spectrum build
// Column pass of the 2D transforms of the coil maps (the row pass already ran
// into `coil_rows`): P = sum_c |DFT(s_c)|^2 (unnormalised) and the pixel coil
// energy sum_c |S_c|^2 (for the Jacobi diagonal).
template <int M>
__global__ __launch_bounds__(ColCfg<M>::THREADS) void k_col_power2d(Ws w, const float2* __restrict__ coil_rows,
                                                                     float* __restrict__ P, float* __restrict__ energy) {
  constexpr int NT = ColCfg<M>::NT, E = ColCfg<M>::E, T = ColCfg<M>::T;
  __shared__ float2 lds[ColLay<T>::template size<M>];
  __shared__ float2 s_tw[M];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  const int n = sd.n;
  const int j = threadIdx.x % T, t = threadIdx.x / T;
  const int col = blockIdx.x * T + j;
  stage_twiddles<M, ColCfg<M>::THREADS>(s_tw, w.tw);
  double pw[E];
  float en[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    pw[e] = 0.0;
    en[e] = 0.f;
  }
  const long long plane = (long long)M * n;
  for (int c = 0; c < sd.nc; ++c) {
    const long long cb = sd.coil + c * plane + col;
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      v[e] = coil_rows[cb + (long long)(t + NT * e) * n];
      en[e] += cabs2(w.sens[cb + (long long)(t + NT * e) * n]);
    }
    fft<M, -1, ColLay<T>>(v, t, lds, j, s_tw);
#pragma unroll
    for (int e = 0; e < E; ++e) pw[e] += (double)v[e].x * v[e].x + (double)v[e].y * v[e].y;
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const long long o = sd.img + (long long)(t + NT * e) * n + col;
    P[o] = (float)pw[e];
    energy[o] = en[e];
  }
}

// a <- mask (as complex), b <- P (as complex); 2D-mask slices only
__global__ __launch_bounds__(256) void k_corr_prep(Ws w, const float* __restrict__ P, float2* __restrict__ a,
                                                   float2* __restrict__ b) {
  const SliceDev sd = w.sl[blockIdx.y];
  if (sd.mask_kind != 1) return;
  const long long np = (long long)sd.m * sd.n;
  const uint8_t* mk = w.mask + sd.mask;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < np; p += (long long)gridDim.x * blockDim.x) {
    a[sd.img + p] = make_float2(mk[p] ? 1.f : 0.f, 0.f);
    b[sd.img + p] = make_float2(P[sd.img + p], 0.f);
  }
}

// a <- a conj(b) after both forward transforms.  The mask transform's DC
// value, the sample count |Omega| (a sum of ones, exact in FP32), is kept in
// the slice's auxiliary partial slot for the Jacobi diagonal.
__global__ __launch_bounds__(256) void k_corr_mul(Ws w, float2* __restrict__ a, const float2* __restrict__ b) {
  const int s = blockIdx.y;
  const SliceDev sd = w.sl[s];
  if (sd.mask_kind != 1) return;
  const long long np = (long long)sd.m * sd.n;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < np; p += (long long)gridDim.x * blockDim.x) {
    const float2 x = a[sd.img + p];
    if (p == 0) part_ptr(w.part, s, P_AUX)[0] = (double)x.x;
    a[sd.img + p] = cconjmul(b[sd.img + p], x);  // x conj(b)
  }
}

// k = mu k_c + lam k_d + gam from the inverse-transformed correlation
// (Re(a) / N^3), optional correction; 1 / (k N) and the Jacobi inverse diagonal.
__global__ __launch_bounds__(256) void k_build_k2d(Ws w, const float2* __restrict__ a, const float* __restrict__ corr,
                                                   const float* __restrict__ energy, float* __restrict__ kraw,
                                                   float* __restrict__ kinv, float* __restrict__ jac,
                                                   int* __restrict__ bad) {
  const int s = blockIdx.y;
  const SliceDev sd = w.sl[s];
  if (sd.mask_kind != 1) return;
  const int m = sd.m, n = sd.n;
  const double N = (double)m * n;
  const double frac = part_ptr(w.part, s, P_AUX)[0] / N;
  const long long np = (long long)m * n;
  int badl = 0;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < np; p += (long long)gridDim.x * blockDim.x) {
    const int u = int(p / n), v = int(p % n);
    const double kc = (double)a[sd.img + p].x / (N * N * N);
    double k = (double)sd.mu * kc + (double)sd.lam * (4.0 - 2.0 * cospi(2.0 * u / m) - 2.0 * cospi(2.0 * v / n)) +
               (double)sd.gam;
    if (corr) k *= (double)corr[sd.img + p];
    if (!(k > 0.0) || !isfinite(k)) badl = 1;
    kraw[sd.img + p] = (float)k;
    kinv[sd.img + p] = (float)(1.0 / (k * N));
    const double dA = (double)sd.mu * frac * (double)energy[sd.img + p] + 4.0 * sd.lam + sd.gam;
    jac[sd.img + p] = (float)(1.0 / dA);
  }
  if (badl) atomicOr(bad, 1);
}

// ============================================================== launchers

#define PICS_2D_SIZES(X) X(64) X(128) X(192) X(224) X(256) X(320) X(512) X(1024)

hipError_t launch_apply2d(const Launch& L, const Ws& w, int mode, int terms, int pk, double tol, const float2* xin,
                          const float2* zsrc, const float2* pold, float2* pn, float2* out, float2* coil) {
  const bool data = (terms & TERM_DATA) != 0;
  if (mode == CA_PCG && !data) return hipErrorInvalidValue;  // the PCG mode always carries the data term
  const dim3 rgrid(L.m / kRowRR, L.count), cgrid(L.n / col_tile(L.m), L.count);
  if (data) {
    switch (L.n) {
#define PICS_CASE(N)                                                                                             \
  case N:                                                                                                        \
    if (mode == CA_PCG)                                                                                          \
      hipLaunchKernelGGL((k_row_sp<N, CA_PCG>), rgrid, dim3(RowCfg<N>::THREADS), 0, L.stream, w, pk, tol, xin,   \
                         zsrc, pold, pn, coil);                                                                  \
    else                                                                                                         \
      hipLaunchKernelGGL((k_row_sp<N, CA_APPLY>), rgrid, dim3(RowCfg<N>::THREADS), 0, L.stream, w, pk, tol, xin, \
                         zsrc, pold, pn, coil);                                                                  \
    break;
      PICS_2D_SIZES(PICS_CASE)
#undef PICS_CASE
      default:
        return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (L.m) {
#define PICS_CASE(M)                                                                                          \
  case M:                                                                                                     \
    hipLaunchKernelGGL(k_col_mask2d<M>, cgrid, dim3(ColCfg<M>::THREADS), 0, L.stream, w, mode == CA_PCG ? 1 : 0, \
                       coil);                                                                                 \
    break;
      PICS_2D_SIZES(PICS_CASE)
#undef PICS_CASE
      default:
        return hipErrorInvalidValue;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  switch (L.n) {
#define PICS_CASE(N)                                                                                            \
  case N:                                                                                                       \
    if (mode == CA_PCG)                                                                                         \
      hipLaunchKernelGGL((k_row_acc<N, CA_PCG>), rgrid, dim3(RowCfg<N>::THREADS), 0, L.stream, w, terms, xin,   \
                         pn, coil, out);                                                                        \
    else                                                                                                        \
      hipLaunchKernelGGL((k_row_acc<N, CA_APPLY>), rgrid, dim3(RowCfg<N>::THREADS), 0, L.stream, w, terms, xin, \
                         pn, coil, out);                                                                        \
    break;
    PICS_2D_SIZES(PICS_CASE)
#undef PICS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_col_power2d(const Launch& L, const Ws& w, const float2* coil_rows, float* P, float* energy) {
  const dim3 grid(L.n / col_tile(L.m), L.count);
  switch (L.m) {
#define PICS_CASE(M)                                                                                         \
  case M:                                                                                                    \
    hipLaunchKernelGGL(k_col_power2d<M>, grid, dim3(ColCfg<M>::THREADS), 0, L.stream, w, coil_rows, P, energy); \
    break;
    PICS_2D_SIZES(PICS_CASE)
#undef PICS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static dim3 pixel_grid(const Simple& S) {
  long long blocks = (S.max_pixels + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  return dim3((unsigned)std::max(1LL, blocks), S.nslices);
}

hipError_t launch_corr_prep(const Simple& S, const Ws& w, const float* P, float2* a, float2* b) {
  hipLaunchKernelGGL(k_corr_prep, pixel_grid(S), dim3(256), 0, S.stream, w, P, a, b);
  return hipGetLastError();
}

hipError_t launch_corr_mul(const Simple& S, const Ws& w, float2* a, const float2* b) {
  hipLaunchKernelGGL(k_corr_mul, pixel_grid(S), dim3(256), 0, S.stream, w, a, b);
  return hipGetLastError();
}

hipError_t launch_build_k2d(const Simple& S, const Ws& w, const float2* a, const float* corr, const float* energy,
                            float* kraw, float* kinv, float* jac, int* bad) {
  hipLaunchKernelGGL(k_build_k2d, pixel_grid(S), dim3(256), 0, S.stream, w, a, corr, energy, kraw, kinv, jac, bad);
  return hipGetLastError();
}

}  // namespace pics

// Element-wise and reduction kernels of the 3D extension (volume [p][m][n],
// axis 0 = z).  The 3D transforms themselves reuse the row and column FFT
// kernels through slice tables that view a volume as p planes of m x n (row
// and column passes) and as one [p][m n] array (the z pass).
#include "tiles.hpp"

namespace pics {

constexpr int kVolBlocks = kVolDotBlocks;  // blocks of the FP64 dot-product partials

static dim3 vol_grid(long long count) {
  long long b = (count + 255) / 256;
  if (b > 4096) b = 4096;
  return dim3((unsigned)(b < 1 ? 1 : b));
}

// out[c][v] = S[c][v] x[v]
__global__ __launch_bounds__(256) void k3_coil_mul(const float2* __restrict__ S, const float2* __restrict__ x,
                                                   float2* __restrict__ out, int nc, long long V) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nc * V; i += (long long)gridDim.x * blockDim.x)
    out[i] = cmul(S[i], x[i % V]);
}

// buf[c][v] *= r(v) / N (the unitary pair's scale folded into the mask)
__global__ __launch_bounds__(256) void k3_mask_scale(float2* __restrict__ buf, const uint8_t* __restrict__ mask, int nc,
                                                     long long V, float scale) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nc * V; i += (long long)gridDim.x * blockDim.x)
    buf[i] = cscale(buf[i], mask[i % V] ? scale : 0.f);
}

// y = mu sum_c conj(S_c) buf_c + lam (D_z^H D_z + D_y^H D_y + D_x^H D_x) x + gam x
__global__ __launch_bounds__(256) void k3_accumulate(const float2* __restrict__ S, const float2* __restrict__ buf,
                                                     const float2* __restrict__ x, float2* __restrict__ y, int nc, int p,
                                                     int m, int n, float mu, float lam, float gam, int data) {
  const long long V = (long long)p * m * n;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x) {
    float2 acc = make_float2(0.f, 0.f);
    if (data)
      for (int c = 0; c < nc; ++c) acc = cadd(acc, cconjmul(S[c * V + v], buf[c * V + v]));
    const int w = int(v / ((long long)m * n)), u = int((v / n) % m), j = int(v % n);
    const long long pl = (long long)m * n;
    const float2 xc = x[v];
    const float2 nb[6] = {x[(long long)((w + 1) % p) * pl + (long long)u * n + j],
                          x[(long long)((w - 1 + p) % p) * pl + (long long)u * n + j],
                          x[(long long)w * pl + (long long)((u + 1) % m) * n + j],
                          x[(long long)w * pl + (long long)((u - 1 + m) % m) * n + j],
                          x[(long long)w * pl + (long long)u * n + (j + 1) % n],
                          x[(long long)w * pl + (long long)u * n + (j - 1 + n) % n]};
    float2 lap = make_float2(6.f * xc.x, 6.f * xc.y);
#pragma unroll
    for (int k = 0; k < 6; ++k) lap = csub(lap, nb[k]);
    y[v] = make_float2(mu * acc.x + lam * lap.x + gam * xc.x, mu * acc.y + lam * lap.y + gam * xc.y);
  }
}

// P[v] = sum_c |buf_c[v]|^2 (buf: the coil maps' unnormalised 3D transforms)
__global__ __launch_bounds__(256) void k3_power(const float2* __restrict__ buf, float* __restrict__ P, int nc,
                                                long long V) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x) {
    double a = 0.0;
    for (int c = 0; c < nc; ++c) {
      const float2 z = buf[c * V + v];
      a += (double)z.x * z.x + (double)z.y * z.y;
    }
    P[v] = (float)a;
  }
}

__global__ __launch_bounds__(256) void k3_corr_prep(const uint8_t* __restrict__ mask, const float* __restrict__ P,
                                                    float2* __restrict__ a, float2* __restrict__ b, long long V) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x) {
    a[v] = make_float2(mask[v] ? 1.f : 0.f, 0.f);
    b[v] = make_float2(P[v], 0.f);
  }
}

// a <- a conj(b); a's DC value (the sample count, exact) is not needed here
__global__ __launch_bounds__(256) void k3_corr_mul(float2* __restrict__ a, const float2* __restrict__ b, long long V) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x)
    a[v] = cconjmul(b[v], a[v]);
}

// k = mu Re(a) / N^3 + lam k_d + gam, 1 / (k N)
__global__ __launch_bounds__(256) void k3_build_k(const float2* __restrict__ a, float* __restrict__ kraw,
                                                  float* __restrict__ kinv, int* __restrict__ bad, int p, int m, int n,
                                                  double mu, double lam, double gam) {
  const long long V = (long long)p * m * n;
  const double N = (double)V;
  int badl = 0;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x) {
    const int w = int(v / ((long long)m * n)), u = int((v / n) % m), j = int(v % n);
    const double kd = 6.0 - 2.0 * cospi(2.0 * w / p) - 2.0 * cospi(2.0 * u / m) - 2.0 * cospi(2.0 * j / n);
    const double k = mu * ((double)a[v].x / (N * N * N)) + lam * kd + gam;
    if (!(k > 0.0) || !isfinite(k)) badl = 1;
    kraw[v] = (float)k;
    kinv[v] = (float)(1.0 / (k * N));
  }
  if (badl) atomicOr(bad, 1);
}

__global__ __launch_bounds__(256) void k3_scale(float2* __restrict__ buf, const float* __restrict__ s, long long V) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x)
    buf[v] = cscale(buf[v], s[v]);
}

// ----------------------------------------------------------------------------
// Operator for masks that are constant along x (axis 2; the generators' 2D
// variable-density pattern over (z, y) with x fully sampled).  Then the 3D
// data term factors as F^H R F = (F_zy^H R_zy F_zy) (x) I_x: each coil needs
// transforms along y and z only, and x is the contiguous batch axis of every
// pass.  The x axis is taken in chunks of X columns (x0 .. x0 + X - 1); each
// chunk runs three passes over a chunk workspace [nc][p][m][X]:
//   1. y-columns of each plane:  u_c = F_y (S_c x)                     (k3_col_sp)
//   2. z-columns of each coil:   u_c = F_z^H (r / (p m)) F_z u_c        (k3_col_z)
//   3. y-columns of each plane:  y = mu sum_c conj(S_c) F_y^H u_c
//                                    + lam (D_z^H D_z + D_y^H D_y + D_x^H D_x) x + gam x  (k3_col_acc)
// A chunk's workspace is sized to stay in the last-level cache between its
// passes (the next chunk reuses the same lines).  Each column workgroup owns
// T adjacent x columns of one plane (passes 1, 3) or of the flattened (y, x)
// index of the chunk (pass 2) and the whole transform length.
// ----------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(ColCfg<M>::THREADS) void k3_col_sp(const float2* __restrict__ S,
                                                                const float2* __restrict__ x,
                                                                float2* __restrict__ coil,
                                                                const float2* __restrict__ tw, int nc, int n,
                                                                long long V, int x0, int X) {
  constexpr int NT = ColCfg<M>::NT, E = ColCfg<M>::E, T = ColCfg<M>::T, TH = ColCfg<M>::THREADS;
  __shared__ float2 lds[ColLay<T>::template size<M>];
  __shared__ float2 s_tw[M];
  const int j = threadIdx.x % T, t = threadIdx.x / T;
  const int jc = xcd_tile(blockIdx.x, gridDim.x) * T + j;  // column within the chunk
  const long long base = (long long)blockIdx.y * M * n + x0 + jc + (long long)t * n;
  const long long VC = (long long)gridDim.y * M * X;  // one coil's chunk workspace
  const long long cbase = (long long)blockIdx.y * M * X + jc + (long long)t * X;
  stage_twiddles<M, TH>(s_tw, tw);
  float2 xv[E], sv[E], sn[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    xv[e] = x[base + (long long)NT * e * n];
    sv[e] = S[base + (long long)NT * e * n];
  }
  for (int c = 0; c < nc; ++c) {
    const long long off = (long long)c * V + base;
    // the next coil's maps are loaded while this coil is transformed
    // (unconditional: the last trip reloads its own)
    const long long nx = c + 1 < nc ? V : 0;
#pragma unroll
    for (int e = 0; e < E; ++e) sn[e] = S[off + nx + (long long)NT * e * n];
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cmul(sv[e], xv[e]);
    fft<M, -1, ColLay<T>>(v, t, lds, j, s_tw);
    float2* __restrict__ o = coil + (long long)c * VC + cbase;
#pragma unroll
    for (int e = 0; e < E; ++e) o[(long long)NT * e * X] = v[e];
#pragma unroll
    for (int e = 0; e < E; ++e) sv[e] = sn[e];
  }
}

// grid.y = coil; the chunk workspace of one coil is [P][m][X], a z-column is
// one (y, x) index of the chunk
template <int P>
__global__ __launch_bounds__(ColCfg<P>::THREADS) void k3_col_z(float2* __restrict__ coil,
                                                               const uint8_t* __restrict__ mask,
                                                               const float2* __restrict__ tw, int n, int x0, int X,
                                                               long long mX, float scale) {
  constexpr int NT = ColCfg<P>::NT, E = ColCfg<P>::E, T = ColCfg<P>::T, TH = ColCfg<P>::THREADS;
  __shared__ float2 lds[ColLay<T>::template size<P>];
  __shared__ float2 s_tw[P];
  const int j = threadIdx.x % T, t = threadIdx.x / T;
  const long long col = (long long)xcd_tile(blockIdx.x, gridDim.x) * T + j;  // (y, x) index in the chunk
  const long long mn = mX / X * n;                                           // one plane of the mask
  const long long mcol = (col / X) * n + x0 + col % X;                       // the same index in the mask
  float2* __restrict__ cb = coil + (long long)blockIdx.y * P * mX + col;
  stage_twiddles<P, TH>(s_tw, tw);
  float2 v[E];
  float sc[E];  // r(z, y) / (p m): the pair's scale folded into the mask
#pragma unroll
  for (int e = 0; e < E; ++e) {
    v[e] = cb[(long long)(t + NT * e) * mX];
    sc[e] = mask[(long long)(t + NT * e) * mn + mcol] ? scale : 0.f;
  }
  fft<P, -1, ColLay<T>>(v, t, lds, j, s_tw);
  fft_in_scaled<P, +1, ColLay<T>, false>(v, sc, t, lds, lds, j, s_tw);
#pragma unroll
  for (int e = 0; e < E; ++e) cb[(long long)(t + NT * e) * mX] = v[e];
}

template <int M>
struct Acc3Cfg {
  static constexpr int T = ColCfg<M>::T;
  static constexpr int TS = T + 2;  // tile stride with the two halo x columns
  static constexpr int LB = ColLay<T>::template size<M>;
  static constexpr int LDS = LB > M * TS ? LB : M * TS;
};

template <int M>
__global__ __launch_bounds__(ColCfg<M>::THREADS) void k3_col_acc(const float2* __restrict__ S,
                                                                 const float2* __restrict__ coil,
                                                                 const float2* __restrict__ x, float2* __restrict__ y,
                                                                 const float2* __restrict__ tw, int nc, int p, int n,
                                                                 long long V, float mu, float lam, float gam,
                                                                 int data, int x0, int X) {
  constexpr int NT = ColCfg<M>::NT, E = ColCfg<M>::E, T = ColCfg<M>::T, TH = ColCfg<M>::THREADS;
  constexpr int TS = Acc3Cfg<M>::TS;
  __shared__ float2 lds[Acc3Cfg<M>::LDS];
  __shared__ float2 s_tw[M];
  const int j = threadIdx.x % T, t = threadIdx.x / T;
  const int w = blockIdx.y;
  const int jc0 = xcd_tile(blockIdx.x, gridDim.x) * T;  // tile start within the chunk
  const int j0 = x0 + jc0;                              // and in the volume
  const long long pl = (long long)M * n;
  const long long base = (long long)w * pl + j0 + j + (long long)t * n;
  const long long VC = (long long)p * M * X;
  const long long cbase = (long long)w * M * X + jc0 + j + (long long)t * X;
  stage_twiddles<M, TH>(s_tw, tw);
  float2 acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = make_float2(0.f, 0.f);
  if (data) {
    // the next coil's column and maps are loaded while this coil is transformed
    float2 v[E], vn[E], sv[E], sn[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      v[e] = coil[cbase + (long long)NT * e * X];
      sv[e] = S[base + (long long)NT * e * n];
    }
    for (int c = 0; c < nc; ++c) {
      const int cn = c + 1 < nc ? c + 1 : c;
      const long long nx = (long long)cn * V + base, ncx = (long long)cn * VC + cbase;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        vn[e] = coil[ncx + (long long)NT * e * X];
        sn[e] = S[nx + (long long)NT * e * n];
      }
      fft<M, +1, ColLay<T>>(v, t, lds, j, s_tw);
#pragma unroll
      for (int e = 0; e < E; ++e) acc[e] = cadd(acc[e], cconjmul(sv[e], v[e]));
#pragma unroll
      for (int e = 0; e < E; ++e) {
        v[e] = vn[e];
        sv[e] = sn[e];
      }
    }
    __syncthreads();  // the transforms are done with the LDS buffer
  }
  // x on the plane's tile with one halo column on each side (periodic in x)
  for (int k = threadIdx.x; k < M * TS; k += TH) {
    const int u = k / TS, jj = k % TS;
    const int gj = (j0 - 1 + jj + n) % n;
    lds[k] = x[(long long)w * pl + (long long)u * n + gj];
  }
  __syncthreads();
  const long long wu = (long long)((w + 1) % p) * pl, wd = (long long)((w - 1 + p) % p) * pl;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int u = t + NT * e;
    const float2 c0 = lds[u * TS + j + 1];
    const float2 up = lds[((u + 1) % M) * TS + j + 1], dn = lds[((u - 1 + M) % M) * TS + j + 1];
    const float2 l = lds[u * TS + j], r = lds[u * TS + j + 2];
    const long long o = (long long)u * n + j0 + j;
    const float2 zu = x[wu + o], zd = x[wd + o];
    const float2 lap = make_float2(6.f * c0.x - up.x - dn.x - l.x - r.x - zu.x - zd.x,
                                   6.f * c0.y - up.y - dn.y - l.y - r.y - zu.y - zd.y);
    y[(long long)w * pl + o] = make_float2(mu * acc[e].x + lam * lap.x + gam * c0.x,
                                           mu * acc[e].y + lam * lap.y + gam * c0.y);
  }
}

// flag |= 1 if the mask [rows][n] is not constant along its last axis
__global__ __launch_bounds__(256) void k3_xconst(const uint8_t* __restrict__ mask, long long rows, int n,
                                                 int* __restrict__ flag) {
  int bad = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < rows * n; i += (long long)gridDim.x * blockDim.x)
    if ((mask[i] != 0) != (mask[(i / n) * n] != 0)) bad = 1;
  if (bad) atomicOr(flag, 1);
}

// ---------------------------------------------------------------- PCG
// part[slot][block] = sum over the block's voxels of Re(conj(a) b) (FP64)
__global__ __launch_bounds__(256) void k3_dot(const float2* __restrict__ a, const float2* __restrict__ b, long long V,
                                              double* __restrict__ part, int slot) {
  __shared__ double red[16];
  double acc = 0.0;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x)
    acc += (double)a[v].x * b[v].x + (double)a[v].y * b[v].y;
  acc = block_sum_f64(acc, red);
  if (threadIdx.x == 0) part[slot * kVolBlocks + blockIdx.x] = acc;
}

// scal[idx] = sum of the slot's partials in block order (one thread)
__global__ void k3_finish_dot(const double* __restrict__ part, int slot, double* __restrict__ scal, int idx) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double a = 0.0;
    for (int b = 0; b < kVolBlocks; ++b) a += part[slot * kVolBlocks + b];
    scal[idx] = a;
  }
}

// r = b - q
__global__ __launch_bounds__(256) void k3_residual(const float2* __restrict__ b, const float2* __restrict__ q,
                                                   float2* __restrict__ r, long long V) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x)
    r[v] = csub(b[v], q[v]);
}

// alpha = scal[irho] / scal[isig]; x += alpha p; r -= alpha q
__global__ __launch_bounds__(256) void k3_update_xr(float2* __restrict__ x, float2* __restrict__ r,
                                                    const float2* __restrict__ p, const float2* __restrict__ q,
                                                    const double* __restrict__ scal, int irho, int isig, long long V) {
  const float al = (float)(scal[irho] / scal[isig]);
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x) {
    const float2 pv = p[v], qv = q[v];
    x[v] = make_float2(x[v].x + al * pv.x, x[v].y + al * pv.y);
    r[v] = make_float2(r[v].x - al * qv.x, r[v].y - al * qv.y);
  }
}

// beta = scal[inew] / scal[iold] (0 when iold < 0); p = z + beta p
__global__ __launch_bounds__(256) void k3_update_p(float2* __restrict__ p, const float2* __restrict__ z,
                                                   const double* __restrict__ scal, int inew, int iold, long long V) {
  const float be = iold < 0 ? 0.f : (float)(scal[inew] / scal[iold]);
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x) {
    const float2 pv = p[v], zv = z[v];
    p[v] = make_float2(zv.x + be * pv.x, zv.y + be * pv.y);
  }
}

// ============================================================== launchers

hipError_t launch3_coil_mul(hipStream_t st, const float2* S, const float2* x, float2* out, int nc, long long V) {
  hipLaunchKernelGGL(k3_coil_mul, vol_grid(nc * V), dim3(256), 0, st, S, x, out, nc, V);
  return hipGetLastError();
}
hipError_t launch3_mask_scale(hipStream_t st, float2* buf, const uint8_t* mask, int nc, long long V, float scale) {
  hipLaunchKernelGGL(k3_mask_scale, vol_grid(nc * V), dim3(256), 0, st, buf, mask, nc, V, scale);
  return hipGetLastError();
}
hipError_t launch3_accumulate(hipStream_t st, const float2* S, const float2* buf, const float2* x, float2* y, int nc,
                              int p, int m, int n, float mu, float lam, float gam, int data) {
  hipLaunchKernelGGL(k3_accumulate, vol_grid((long long)p * m * n), dim3(256), 0, st, S, buf, x, y, nc, p, m, n, mu,
                     lam, gam, data);
  return hipGetLastError();
}
hipError_t launch3_power(hipStream_t st, const float2* buf, float* P, int nc, long long V) {
  hipLaunchKernelGGL(k3_power, vol_grid(V), dim3(256), 0, st, buf, P, nc, V);
  return hipGetLastError();
}
hipError_t launch3_corr_prep(hipStream_t st, const uint8_t* mask, const float* P, float2* a, float2* b, long long V) {
  hipLaunchKernelGGL(k3_corr_prep, vol_grid(V), dim3(256), 0, st, mask, P, a, b, V);
  return hipGetLastError();
}
hipError_t launch3_corr_mul(hipStream_t st, float2* a, const float2* b, long long V) {
  hipLaunchKernelGGL(k3_corr_mul, vol_grid(V), dim3(256), 0, st, a, b, V);
  return hipGetLastError();
}
hipError_t launch3_build_k(hipStream_t st, const float2* a, float* kraw, float* kinv, int* bad, int p, int m, int n,
                           double mu, double lam, double gam) {
  hipLaunchKernelGGL(k3_build_k, vol_grid((long long)p * m * n), dim3(256), 0, st, a, kraw, kinv, bad, p, m, n, mu,
                     lam, gam);
  return hipGetLastError();
}
hipError_t launch3_scale(hipStream_t st, float2* buf, const float* s, long long V) {
  hipLaunchKernelGGL(k3_scale, vol_grid(V), dim3(256), 0, st, buf, s, V);
  return hipGetLastError();
}
hipError_t launch3_dot(hipStream_t st, const float2* a, const float2* b, long long V, double* part, int slot,
                       double* scal, int idx) {
  hipLaunchKernelGGL(k3_dot, dim3(kVolBlocks), dim3(256), 0, st, a, b, V, part, slot);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k3_finish_dot, dim3(1), dim3(64), 0, st, part, slot, scal, idx);
  return hipGetLastError();
}
hipError_t launch3_residual(hipStream_t st, const float2* b, const float2* q, float2* r, long long V) {
  hipLaunchKernelGGL(k3_residual, vol_grid(V), dim3(256), 0, st, b, q, r, V);
  return hipGetLastError();
}
hipError_t launch3_update_xr(hipStream_t st, float2* x, float2* r, const float2* p, const float2* q, const double* scal,
                             int irho, int isig, long long V) {
  hipLaunchKernelGGL(k3_update_xr, vol_grid(V), dim3(256), 0, st, x, r, p, q, scal, irho, isig, V);
  return hipGetLastError();
}
hipError_t launch3_update_p(hipStream_t st, float2* p, const float2* z, const double* scal, int inew, int iold,
                            long long V) {
  hipLaunchKernelGGL(k3_update_p, vol_grid(V), dim3(256), 0, st, p, z, scal, inew, iold, V);
  return hipGetLastError();
}


hipError_t launch3_col_sp(hipStream_t st, const float2* S, const float2* x, float2* coil, const float2* tw, int nc,
                          int p, int m, int n, int x0, int X) {
  const long long V = (long long)p * m * n;
  const dim3 grid(X / col_tile(m), p);
  switch (m) {
#define PICS_CASE(M)                                                                                         \
  case M:                                                                                                    \
    hipLaunchKernelGGL(k3_col_sp<M>, grid, dim3(ColCfg<M>::THREADS), 0, st, S, x, coil, tw, nc, n, V, x0, X); \
    break;
    PICS_FFT_SIZES(PICS_CASE)
#undef PICS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch3_col_z(hipStream_t st, float2* coil, const uint8_t* mask, const float2* tw, int nc, int p, int m,
                         int n, int x0, int X, float scale) {
  const long long mX = (long long)m * X;
  const dim3 grid((unsigned)(mX / col_tile(p)), nc);
  switch (p) {
#define PICS_CASE(P)                                                                                               \
  case P:                                                                                                          \
    hipLaunchKernelGGL(k3_col_z<P>, grid, dim3(ColCfg<P>::THREADS), 0, st, coil, mask, tw, n, x0, X, mX, scale); \
    break;
    PICS_FFT_SIZES(PICS_CASE)
#undef PICS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch3_col_acc(hipStream_t st, const float2* S, const float2* coil, const float2* x, float2* y,
                           const float2* tw, int nc, int p, int m, int n, float mu, float lam, float gam, int data,
                           int x0, int X) {
  const long long V = (long long)p * m * n;
  const dim3 grid(X / col_tile(m), p);
  switch (m) {
#define PICS_CASE(M)                                                                                          \
  case M:                                                                                                     \
    hipLaunchKernelGGL(k3_col_acc<M>, grid, dim3(ColCfg<M>::THREADS), 0, st, S, coil, x, y, tw, nc, p, n, V, \
                       mu, lam, gam, data, x0, X);                                                            \
    break;
    PICS_FFT_SIZES(PICS_CASE)
#undef PICS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch3_xconst(hipStream_t st, const uint8_t* mask, long long rows, int n, int* flag) {
  hipLaunchKernelGGL(k3_xconst, vol_grid(rows * n), dim3(256), 0, st, mask, rows, n, flag);
  return hipGetLastError();
}

}  // namespace pics

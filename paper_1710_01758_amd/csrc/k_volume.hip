// Element-wise and reduction kernels of the 3D extension (volume [p][m][n],
// axis 0 = z).  The 3D transforms themselves reuse the row and column FFT
// kernels through slice tables that view a volume as p planes of m x n (row
// and column passes) and as one [p][m n] array (the z pass).
#include "internal.hpp"

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

}  // namespace pics

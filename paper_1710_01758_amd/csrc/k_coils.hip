// Coil compression (Methods, Coil compression; principal-component channel
// compression): per slice the coil covariance C = sum_k y(k) y(k)^H of the
// acquired samples, its eigen-decomposition by cyclic Jacobi rotations in
// FP64, and the mixing y_v = U_v^H y, S_v = U_v^H S onto the most dominant
// virtual coils.
#include "internal.hpp"

namespace pics {

constexpr int kCovBlocks = 32;   // covariance partials per slice
constexpr int kCovPix = 64;      // pixels per LDS tile
constexpr int kMaxCoils = 32;  // coils per slice accepted by compression

__device__ __forceinline__ double2 dmul_conj(float2 a, float2 b) {  // a conj(b)
  return make_double2((double)a.x * b.x + (double)a.y * b.y, (double)a.y * b.x - (double)a.x * b.y);
}

// partial[blk][i][j] = sum over the block's pixels of y_i conj(y_j)
__global__ __launch_bounds__(256) void k_coil_cov(Ws w, const float2* __restrict__ ksp, double2* __restrict__ scratch) {
  __shared__ float2 tile[kCovPix][kMaxCoils + 1];
  const int s = blockIdx.y;
  const SliceDev sd = w.sl[s];
  const int nc = sd.nc;
  const long long np = (long long)sd.m * sd.n;
  const long long chunk = (np + kCovBlocks - 1) / kCovBlocks;
  const long long p0 = blockIdx.x * chunk, p1 = p0 + chunk < np ? p0 + chunk : np;
  const int npair = nc * nc;
  double2 acc[4] = {};  // pairs threadIdx.x + 256 q (nc <= 32: at most 1024 pairs)
  for (long long base = p0; base < p1; base += kCovPix) {
    __syncthreads();
    for (int k = threadIdx.x; k < kCovPix * nc; k += blockDim.x) {
      const int c = k / kCovPix, px = k % kCovPix;
      const long long p = base + px;
      tile[px][c] = p < p1 ? ksp[sd.coil + (long long)c * np + p] : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int pr = threadIdx.x + 256 * q;
      if (pr < npair) {
        const int i = pr / nc, j = pr % nc;
        double2 a = acc[q];
        for (int px = 0; px < kCovPix; ++px) {
          const double2 v = dmul_conj(tile[px][i], tile[px][j]);
          a.x += v.x;
          a.y += v.y;
        }
        acc[q] = a;
      }
    }
  }
  double2* out = scratch + sd.coil / 2 + (long long)blockIdx.x * npair;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int pr = threadIdx.x + 256 * q;
    if (pr < npair) out[pr] = acc[q];
  }
}

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One wave per slice: reduce the partials in block order, diagonalise C by
// cyclic Jacobi rotations (each zeroes one off-diagonal pair with a unitary
// 2 x 2 transform), sort by descending eigenvalue, write the first nvirt
// eigenvectors (float, [c][v]) after the partials and the eigenvalues into
// the slice's auxiliary partial slot.
__global__ __launch_bounds__(64) void k_coil_eig(Ws w, double2* __restrict__ scratch, int nvirt) {
  __shared__ double2 A[kMaxCoils][kMaxCoils + 1];
  __shared__ double2 V[kMaxCoils][kMaxCoils + 1];
  __shared__ double2 rot[3];  // c, s, e^{-i phi}
  __shared__ int order[kMaxCoils];
  __shared__ double off_s, tot_s;
  const int s = blockIdx.x;
  const SliceDev sd = w.sl[s];
  const int nc = sd.nc, npair = nc * nc, lane = threadIdx.x;
  const double2* part = scratch + sd.coil / 2;
  for (int pr = lane; pr < npair; pr += 64) {
    double2 a = make_double2(0.0, 0.0);
    for (int b = 0; b < kCovBlocks; ++b) {
      a.x += part[(long long)b * npair + pr].x;
      a.y += part[(long long)b * npair + pr].y;
    }
    A[pr / nc][pr % nc] = a;
    V[pr / nc][pr % nc] = make_double2(pr / nc == pr % nc ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (lane == 0) {
      double off = 0.0, tot = 0.0;
      for (int i = 0; i < nc; ++i)
        for (int j = 0; j < nc; ++j) {
          const double v = A[i][j].x * A[i][j].x + A[i][j].y * A[i][j].y;
          tot += v;
          if (i != j) off += v;
        }
      off_s = off;
      tot_s = tot;
    }
    __syncthreads();
    if (!(off_s > 1e-28 * tot_s)) break;
    for (int p = 0; p < nc - 1; ++p)
      for (int q = p + 1; q < nc; ++q) {
        if (lane == 0) {
          const double2 g = A[p][q];
          const double ag = sqrt(g.x * g.x + g.y * g.y);
          if (ag <= 1e-300) {
            rot[0] = make_double2(1.0, 0.0);
            rot[1] = make_double2(0.0, 0.0);
            rot[2] = make_double2(1.0, 0.0);
          } else {
            const double tau = (A[q][q].x - A[p][p].x) / (2.0 * ag);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            const double c = 1.0 / sqrt(1.0 + t * t);
            rot[0] = make_double2(c, 0.0);
            rot[1] = make_double2(t * c, 0.0);
            rot[2] = make_double2(g.x / ag, -g.y / ag);  // e^{-i phi}, phi = arg A_pq
          }
        }
        __syncthreads();
        const double c = rot[0].x, sn = rot[1].x;
        const double2 em = rot[2], ep = make_double2(em.x, -em.y);
        // G = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] on coordinates (p, q)
        if (lane < nc) {  // A <- A G, V <- V G (rows k)
          const int k = lane;
          const double2 akp = A[k][p], akq = zmul(A[k][q], em);
          A[k][p] = make_double2(c * akp.x - sn * akq.x, c * akp.y - sn * akq.y);
          A[k][q] = make_double2(sn * akp.x + c * akq.x, sn * akp.y + c * akq.y);
          const double2 vkp = V[k][p], vkq = zmul(V[k][q], em);
          V[k][p] = make_double2(c * vkp.x - sn * vkq.x, c * vkp.y - sn * vkq.y);
          V[k][q] = make_double2(sn * vkp.x + c * vkq.x, sn * vkp.y + c * vkq.y);
        }
        __syncthreads();
        if (lane < nc) {  // A <- G^H A (columns k)
          const int k = lane;
          const double2 apk = A[p][k], aqk = zmul(A[q][k], ep);
          A[p][k] = make_double2(c * apk.x - sn * aqk.x, c * apk.y - sn * aqk.y);
          A[q][k] = make_double2(sn * apk.x + c * aqk.x, sn * apk.y + c * aqk.y);
        }
        __syncthreads();
        if (lane == 0) {
          A[p][q] = make_double2(0.0, 0.0);
          A[q][p] = make_double2(0.0, 0.0);
          A[p][p].y = 0.0;
          A[q][q].y = 0.0;
        }
        __syncthreads();
      }
  }
  if (lane == 0) {
    for (int i = 0; i < nc; ++i) order[i] = i;
    for (int i = 0; i < nc; ++i) {
      int best = i;
      for (int j = i + 1; j < nc; ++j)
        if (A[order[j]][order[j]].x > A[order[best]][order[best]].x) best = j;
      const int tmp = order[i];
      order[i] = order[best];
      order[best] = tmp;
    }
  }
  __syncthreads();
  double* eig = part_ptr(w.part, s, P_AUX);
  if (lane < nc) eig[lane] = A[order[lane]][order[lane]].x;
  float2* U = reinterpret_cast<float2*>(scratch + sd.coil / 2 + (long long)kCovBlocks * npair);
  for (int k = lane; k < nc * nvirt; k += 64) {
    const int c = k / nvirt, v = k % nvirt;
    const double2 u = V[c][order[v]];
    U[k] = make_float2((float)u.x, (float)u.y);
  }
}

// out[v] = sum_c conj(U[c][v]) in[c] per pixel; `in` coil-packed with the
// slice's coil count, `out` coil-packed with nvirt coils per slice
__global__ __launch_bounds__(256) void k_coil_mix(Ws w, const double2* __restrict__ scratch, int nvirt,
                                                  const float2* __restrict__ in, float2* __restrict__ out) {
  __shared__ float2 U[kMaxCoils * kMaxCoils];
  const int s = blockIdx.y;
  const SliceDev sd = w.sl[s];
  const int nc = sd.nc;
  const long long np = (long long)sd.m * sd.n;
  const float2* Ug = reinterpret_cast<const float2*>(scratch + sd.coil / 2 + (long long)kCovBlocks * nc * nc);
  for (int k = threadIdx.x; k < nc * nvirt; k += blockDim.x) U[k] = Ug[k];
  __syncthreads();
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < np; p += (long long)gridDim.x * blockDim.x) {
    for (int v = 0; v < nvirt; ++v) {  // the coil values are re-read per virtual coil (cache hits)
      float2 a = make_float2(0.f, 0.f);
      for (int c = 0; c < nc; ++c) a = cadd(a, cconjmul(U[c * nvirt + v], in[sd.coil + (long long)c * np + p]));
      out[sd.img * nvirt + (long long)v * np + p] = a;
    }
  }
}

hipError_t launch_coil_compress(const Simple& S, const Ws& w, const float2* ksp, const float2* sens, int nvirt,
                                double2* scratch, float2* ksp_out, float2* sens_out) {
  hipLaunchKernelGGL(k_coil_cov, dim3(kCovBlocks, S.nslices), dim3(256), 0, S.stream, w, ksp, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_coil_eig, dim3(S.nslices), dim3(64), 0, S.stream, w, scratch, nvirt);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  long long blocks = (S.max_pixels + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  const dim3 grid((unsigned)(blocks < 1 ? 1 : blocks), S.nslices);
  hipLaunchKernelGGL(k_coil_mix, grid, dim3(256), 0, S.stream, w, scratch, nvirt, ksp, ksp_out);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_coil_mix, grid, dim3(256), 0, S.stream, w, scratch, nvirt, sens, sens_out);
  return hipGetLastError();
}

}  // namespace pics

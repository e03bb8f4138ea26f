// Coil compression (Methods, Coil compression; principal-component channel
// compression): per slice the coil covariance C = sum_k y(k) y(k)^H of the
// acquired samples, its eigen-decomposition by cyclic Jacobi rotations in
// FP64, and the mixing y_v = U_v^H y, S_v = U_v^H S onto the most dominant
// virtual coils.
#include "internal.hpp"

namespace pics {

constexpr int kCovPix = 64;      // pixels per LDS tile
constexpr int kMaxCoils = 32;    // coils per slice accepted by compression

// Covariance partials per slice: as many as fit the slice's coil workspace
// together with the reduced covariance and the eigenvectors (partials take
// 16 nc^2 bytes each, the workspace 8 nc N), at most 128.
__device__ __host__ __forceinline__ int cov_blocks(long long np, int nc) {
  long long b = np / (4LL * nc) - 2;
  return (int)(b < 1 ? 1 : (b > 128 ? 128 : b));
}

__device__ __forceinline__ double2 dmul_conj(float2 a, float2 b) {  // a conj(b)
  return make_double2((double)a.x * b.x + (double)a.y * b.y, (double)a.y * b.x - (double)a.x * b.y);
}

// partial[blk][i][j] = sum over the block's pixels of y_i conj(y_j).  Line
// masks: 64-pixel tiles within unsampled k-space rows hold zeros and are
// skipped.
__global__ __launch_bounds__(256) void k_coil_cov(Ws w, const float2* __restrict__ ksp, double2* __restrict__ scratch) {
  __shared__ float2 tile[kCovPix][kMaxCoils + 1];
  const int s = blockIdx.y;
  const SliceDev sd = w.sl[s];
  const int nc = sd.nc;
  const long long np = (long long)sd.m * sd.n;
  const int nblk = cov_blocks(np, nc);
  if ((int)blockIdx.x >= nblk) return;
  const long long chunk = ((np + nblk - 1) / nblk + kCovPix - 1) / kCovPix * kCovPix;
  const long long p0 = blockIdx.x * chunk, p1 = p0 + chunk < np ? p0 + chunk : np;
  const uint8_t* mk = w.mask + sd.mask;
  const int npair = nc * nc;
  double2 acc[4] = {};  // pairs threadIdx.x + 256 q (nc <= 32: at most 1024 pairs)
  for (long long base = p0; base < p1; base += kCovPix) {
    if (sd.mask_kind == 0) {  // a tile spans at most two rows (n >= 64): skip it if both are unsampled
      const long long last = (base + kCovPix < p1 ? base + kCovPix : p1) - 1;
      if (!mk[base / sd.n] && !mk[last / sd.n]) continue;
    }
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

// C[pr] = sum of the slice's partials in block order (four interleaved
// accumulators combined in fixed order), written after the partials.
__global__ __launch_bounds__(256) void k_coil_cov_reduce(Ws w, double2* __restrict__ scratch) {
  const int s = blockIdx.y;
  const SliceDev sd = w.sl[s];
  const int nc = sd.nc, npair = nc * nc;
  const int pr = blockIdx.x * blockDim.x + threadIdx.x;
  if (pr >= npair) return;
  const int nblk = cov_blocks((long long)sd.m * sd.n, nc);
  double2* part = scratch + sd.coil / 2;
  double2 a[4] = {};
  int b = 0;
  for (; b + 4 <= nblk; b += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double2 v = part[(long long)(b + u) * npair + pr];
      a[u].x += v.x;
      a[u].y += v.y;
    }
  }
  for (; b < nblk; ++b) {
    const double2 v = part[(long long)b * npair + pr];
    a[0].x += v.x;
    a[0].y += v.y;
  }
  part[(long long)nblk * npair + pr] = make_double2((a[0].x + a[1].x) + (a[2].x + a[3].x),
                                                   (a[0].y + a[1].y) + (a[2].y + a[3].y));
}

// Pair i of round r of a round-robin schedule over n (even) indices: every
// pair occurs once in n - 1 rounds and the pairs of one round are disjoint.
__device__ __forceinline__ void rr_pair(int n, int r, int i, int* p, int* q) {
  int a, b;
  if (i == 0) {
    a = 0;
    b = 1 + r % (n - 1);
  } else {
    a = 1 + (r + i) % (n - 1);
    b = 1 + (r - i + (n - 1)) % (n - 1);
  }
  *p = a < b ? a : b;
  *q = a < b ? b : a;
}

// One workgroup per slice (thread (i, k): rotation pair i, row / column k):
// diagonalise C by Jacobi sweeps (each rotation zeroes one off-diagonal pair
// with the unitary G = [[c, s], [-s e^{-i phi}, c e^{-i phi}]], phi = arg
// C_pq; the disjoint pairs of a round-robin round are rotated together),
// sort by descending eigenvalue, write the first nvirt eigenvectors (float,
// [c][v]) after the reduced covariance and the eigenvalues into the slice's
// auxiliary partial slot.
constexpr int kEigThreads = (kMaxCoils / 2) * kMaxCoils;

__global__ __launch_bounds__(kEigThreads) void k_coil_eig(Ws w, double2* __restrict__ scratch, int nvirt) {
  __shared__ double2 A[kMaxCoils][kMaxCoils + 1];
  __shared__ double2 V[kMaxCoils][kMaxCoils + 1];
  __shared__ double rc[kMaxCoils / 2], rsn[kMaxCoils / 2];
  __shared__ double2 rem[kMaxCoils / 2];
  __shared__ int rp[kMaxCoils / 2], rq[kMaxCoils / 2];
  __shared__ int order[kMaxCoils];
  __shared__ double red_off[kEigThreads / 64], red_tot[kEigThreads / 64];
  const int s = blockIdx.x;
  const SliceDev sd = w.sl[s];
  const int nc = sd.nc, npair = nc * nc, tid = threadIdx.x;
  const long long np = (long long)sd.m * sd.n;
  const int nblk = cov_blocks(np, nc);
  const double2* cov = scratch + sd.coil / 2 + (long long)nblk * npair;
  for (int pr = tid; pr < npair; pr += kEigThreads) {
    A[pr / nc][pr % nc] = cov[pr];
    V[pr / nc][pr % nc] = make_double2(pr / nc == pr % nc ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int n2 = nc + (nc & 1);  // odd counts get a dummy index
  const int npr = n2 / 2;
  const int pi = tid / nc, k = tid % nc;  // this thread's pair and row / column
  const bool active = pi < npr;
  for (int sweep = 0; sweep < 30 && nc > 1; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int pr = tid; pr < npair; pr += kEigThreads) {
      const double2 v = A[pr / nc][pr % nc];
      const double a2 = v.x * v.x + v.y * v.y;
      tot += a2;
      if (pr / nc != pr % nc) off += a2;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o, 64);
      tot += __shfl_xor(tot, o, 64);
    }
    if ((tid & 63) == 0) {
      red_off[tid / 64] = off;
      red_tot[tid / 64] = tot;
    }
    __syncthreads();
    double so = 0.0, st = 0.0;
    for (int q = 0; q < kEigThreads / 64; ++q) {
      so += red_off[q];
      st += red_tot[q];
    }
    __syncthreads();
    if (!(so > 1e-28 * st)) break;  // the same decision in every thread
    for (int r = 0; r < n2 - 1; ++r) {
      if (tid < npr) {
        int p, q;
        rr_pair(n2, r, tid, &p, &q);
        double c = 1.0, sn = 0.0;
        double2 em = make_double2(1.0, 0.0);
        if (q < nc) {
          const double2 g = A[p][q];
          const double ag = sqrt(g.x * g.x + g.y * g.y);
          if (ag > 1e-300) {
            const double tau = (A[q][q].x - A[p][p].x) / (2.0 * ag);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = t * c;
            em = make_double2(g.x / ag, -g.y / ag);
          }
        }
        rp[tid] = p;
        rq[tid] = q;
        rc[tid] = c;
        rsn[tid] = sn;
        rem[tid] = em;
      }
      __syncthreads();
      const int p = active ? rp[pi] : 0, q = active ? rq[pi] : 0;
      const bool rot = active && q < nc && rsn[pi] != 0.0;
      const double c = active ? rc[pi] : 1.0, sn = active ? rsn[pi] : 0.0;
      const double2 em = active ? rem[pi] : make_double2(1.0, 0.0);
      if (rot) {  // A <- A G, V <- V G on row k
        const double2 akp = A[k][p], akq = zmul(A[k][q], em);
        A[k][p] = make_double2(c * akp.x - sn * akq.x, c * akp.y - sn * akq.y);
        A[k][q] = make_double2(sn * akp.x + c * akq.x, sn * akp.y + c * akq.y);
        const double2 vkp = V[k][p], vkq = zmul(V[k][q], em);
        V[k][p] = make_double2(c * vkp.x - sn * vkq.x, c * vkp.y - sn * vkq.y);
        V[k][q] = make_double2(sn * vkp.x + c * vkq.x, sn * vkp.y + c * vkq.y);
      }
      __syncthreads();
      if (rot) {  // A <- G^H A on column k
        const double2 ep = make_double2(em.x, -em.y);
        const double2 apk = A[p][k], aqk = zmul(A[q][k], ep);
        A[p][k] = make_double2(c * apk.x - sn * aqk.x, c * apk.y - sn * aqk.y);
        A[q][k] = make_double2(sn * apk.x + c * aqk.x, sn * apk.y + c * aqk.y);
      }
      __syncthreads();
      if (rot && k == 0) {
        A[p][q] = make_double2(0.0, 0.0);
        A[q][p] = make_double2(0.0, 0.0);
        A[p][p].y = 0.0;
        A[q][q].y = 0.0;
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
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
  if (tid < nc) eig[tid] = A[order[tid]][order[tid]].x;
  float2* U = reinterpret_cast<float2*>(scratch + sd.coil / 2 + (long long)(nblk + 1) * npair);
  for (int e = tid; e < nc * nvirt; e += kEigThreads) {
    const int c = e / nvirt, v = e % nvirt;
    const double2 u = V[c][order[v]];
    U[e] = make_float2((float)u.x, (float)u.y);
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
  const float2* Ug =
      reinterpret_cast<const float2*>(scratch + sd.coil / 2 + (long long)(cov_blocks(np, nc) + 1) * nc * nc);
  for (int k = threadIdx.x; k < nc * nvirt; k += blockDim.x) U[k] = Ug[k];
  __syncthreads();
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < np; p += (long long)gridDim.x * blockDim.x) {
    float2 y[kMaxCoils];  // every coil value of the pixel, loaded once
#pragma unroll
    for (int c = 0; c < kMaxCoils; ++c) y[c] = c < nc ? in[sd.coil + (long long)c * np + p] : make_float2(0.f, 0.f);
    for (int v = 0; v < nvirt; ++v) {
      float2 a = make_float2(0.f, 0.f);
#pragma unroll
      for (int c = 0; c < kMaxCoils; ++c)
        if (c < nc) a = cadd(a, cconjmul(U[c * nvirt + v], y[c]));
      out[sd.img * nvirt + (long long)v * np + p] = a;
    }
  }
}

hipError_t launch_coil_compress(const Simple& S, const Ws& w, const float2* ksp, const float2* sens, int nvirt,
                                double2* scratch, float2* ksp_out, float2* sens_out) {
  hipLaunchKernelGGL(k_coil_cov, dim3(128, S.nslices), dim3(256), 0, S.stream, w, ksp, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_coil_cov_reduce, dim3((kMaxCoils * kMaxCoils + 255) / 256, S.nslices), dim3(256), 0, S.stream,
                     w, scratch);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_coil_eig, dim3(S.nslices), dim3(kEigThreads), 0, S.stream, w, scratch, nvirt);
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

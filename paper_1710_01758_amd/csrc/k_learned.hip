// Learned correction of the circulant spectrum (not in the paper): features,
// a 7-layer CNN on a 64 x 64 frequency grid (forward, backward, Adam) and the
// correction map fed to the spectrum build.
//
// Activations are bf16, NHWC ([image][row][col][channel]); 3x3 convolutions
// with circular padding run as implicit GEMMs on the 16x16x16 bf16 matrix
// cores (FP32 accumulation): forward Y[p][o] = sum_(tap,c) X[p + off(tap)][c] W[o][c][tap],
// backward-data dX[p][c] = sum_(tap,o) G[p - off(tap)][o] W[o][c][tap], and the
// weight gradient dW[o][c][tap] = sum_p G[p][o] X[p + off(tap)][c] with the
// pixels as the inner dimension.
#include <algorithm>

#include "internal.hpp"
#include "learned.hpp"

namespace pics {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ __forceinline__ float softplus_f(float o) { return o > 30.f ? o : log1pf(expf(o)); }
__device__ __forceinline__ float sigmoid_f(float o) { return 1.f / (1.f + expf(-o)); }

// --------------------------------------------------------------- features
// Per slice: fft-shifted, area-pooled 64 x 64 maps of the sampled fraction,
// log(energy / mean), log(k / mean) and three constant planes
// log10(mu / 1e-3), log10(lambda / 4e-3), log10(gamma / 4e-3).
__global__ __launch_bounds__(256) void k_features(Ws w, const float* __restrict__ energy,
                                                  const float* __restrict__ kraw, float* __restrict__ feat) {
  __shared__ double red[16];
  __shared__ double sums[2];
  const int s = blockIdx.x;
  const SliceDev sd = w.sl[s];
  const int m = sd.m, n = sd.n, fm = m / kNetGrid, fn = n / kNetGrid;
  const uint8_t* mk = w.mask + sd.mask;
  float* f = feat + (long long)s * kNetFeat * kNetGrid * kNetGrid;
  constexpr int CELLS = kNetGrid * kNetGrid;
  double se = 0.0, sk = 0.0;
  for (int cell = threadIdx.x; cell < CELLS; cell += blockDim.x) {
    const int a = cell / kNetGrid, b = cell % kNetGrid;
    double pm = 0.0, pe = 0.0, pk = 0.0;
    for (int i = 0; i < fm; ++i) {
      const int u = (a * fm + i - m / 2 + m) % m;
      if (sd.mask_kind == 0) pm += mk[u] ? fn : 0.0;
      for (int jj = 0; jj < fn; ++jj) {
        const int v = (b * fn + jj - n / 2 + n) % n;
        const long long p = sd.img + (long long)u * n + v;
        if (sd.mask_kind != 0) pm += mk[(long long)u * n + v] ? 1.0 : 0.0;
        pe += energy[p];
        pk += kraw[p];
      }
    }
    f[0 * CELLS + cell] = (float)(pm / (fm * fn));
    f[1 * CELLS + cell] = (float)(pe / (fm * fn));
    f[2 * CELLS + cell] = (float)(pk / (fm * fn));
    se += pe / (fm * fn);
    sk += pk / (fm * fn);
  }
  se = block_sum_f64(se, red);
  if (threadIdx.x == 0) sums[0] = se / CELLS;
  sk = block_sum_f64(sk, red);
  if (threadIdx.x == 0) sums[1] = sk / CELLS;
  __syncthreads();
  const float lmu = log10f(sd.mu / 1e-3f), llam = log10f(sd.lam / 4e-3f), lgam = log10f(sd.gam / 4e-3f);
  for (int cell = threadIdx.x; cell < CELLS; cell += blockDim.x) {
    f[1 * CELLS + cell] = (float)log((double)f[1 * CELLS + cell] / sums[0] + 1e-6);
    f[2 * CELLS + cell] = (float)log((double)f[2 * CELLS + cell] / sums[1]);
    f[3 * CELLS + cell] = lmu;
    f[4 * CELLS + cell] = llam;
    f[5 * CELLS + cell] = lgam;
  }
}

// ------------------------------------------------------------ network I/O

// features [slice][6][64][64] (FP32) -> X0 [b][64][64][16] (bf16, channels >= 6 zero)
__global__ __launch_bounds__(256) void k_net_input(const float* __restrict__ feat, const int* __restrict__ index,
                                                   uint16_t* __restrict__ x0) {
  const int b = blockIdx.y;
  const int src = index ? index[b] : b;
  constexpr int CELLS = kNetGrid * kNetGrid;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < CELLS * 16; q += gridDim.x * blockDim.x) {
    const int cell = q / 16, c = q % 16;
    const float v = c < kNetFeat ? feat[((long long)src * kNetFeat + c) * CELLS + cell] : 0.f;
    x0[((long long)b * CELLS + cell) * 16 + c] = f2bf(v);
  }
}

// FP32 flat parameters -> bf16 weights in the two GEMM layouts:
// wf[o][tap][cp] (forward B operand) and wb[cp][tap][o] (backward-data B operand),
// cp = padded input channel (zero beyond the real count).
__global__ __launch_bounds__(256) void k_net_prep(const float* __restrict__ theta, NetLayout L) {
  const int l = blockIdx.y;
  const NetLayer& ly = L.layer[l];
  const int total = ly.cout * 9 * ly.cinp;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
    const int o = q / (9 * ly.cinp), r = q % (9 * ly.cinp), tap = r / ly.cinp, cp = r % ly.cinp;
    const float v = cp < ly.cin ? theta[ly.woff + ((long long)o * ly.cin + cp) * 9 + tap] : 0.f;
    const uint16_t h = f2bf(v);
    ly.wf[((long long)o * 9 + tap) * ly.cinp + cp] = h;
    ly.wb[((long long)cp * 9 + tap) * ly.cout + o] = h;
  }
}

// ----------------------------------------------------------- convolutions
// One workgroup = one image row (64 pixels); wave wv owns pixels 16 wv .. 16 wv + 15.
// Lane l: A operand = pixel (l % 16), channels 4 (l / 16) .. +3 of a 16-channel
// chunk; B operand = output channel (l % 16) of a 16-wide tile, same channels;
// result D[4 (l / 16) + i][l % 16].

template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t* __restrict__ x, const uint16_t* __restrict__ wf,
                                                  const float* __restrict__ bias, int dil,
                                                  uint16_t* __restrict__ y) {
  constexpr int G = kNetGrid, NT = COUT / 16, NC = CIN / 16;
  const int b = blockIdx.y, row = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int px = wv * 16 + (lane & 15), kq = (lane >> 4) * 4;
  floatx4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const uint16_t* xb = x + (long long)b * G * G * CIN;
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int ny = (row + dil * (tap / 3 - 1) + 4 * G) % G;
    const int nx = (px + dil * (tap % 3 - 1) + 4 * G) % G;
    const uint16_t* xp = xb + ((long long)ny * G + nx) * CIN + kq;
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) {
      const bf16x4 a = *(const bf16x4*)(xp + ch * 16);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const bf16x4 bw = *(const bf16x4*)(wf + ((long long)(t * 16 + (lane & 15)) * 9 + tap) * CIN + ch * 16 + kq);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw, acc[t], 0, 0, 0);
      }
    }
  }
  uint16_t* yb = y + ((long long)b * G + row) * G * COUT;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int o = t * 16 + (lane & 15);
    const float bo = bias[o];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = wv * 16 + (lane >> 4) * 4 + i;
      yb[(long long)p * COUT + o] = f2bf(fmaxf(acc[t][i] + bo, 0.f));
    }
  }
}

// gprev[p][c] = (xact[p][c] > 0) * sum_(tap,o) g[p - off(tap)][o] W[o][c][tap]
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_bwd_data(const uint16_t* __restrict__ g, const uint16_t* __restrict__ wb,
                                                       const uint16_t* __restrict__ xact, int dil,
                                                       uint16_t* __restrict__ gprev) {
  constexpr int G = kNetGrid, NT = CIN / 16, NC = COUT / 16;
  const int b = blockIdx.y, row = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int px = wv * 16 + (lane & 15), kq = (lane >> 4) * 4;
  floatx4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const uint16_t* gb = g + (long long)b * G * G * COUT;
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int ny = (row - dil * (tap / 3 - 1) + 4 * G) % G;
    const int nx = (px - dil * (tap % 3 - 1) + 4 * G) % G;
    const uint16_t* gp = gb + ((long long)ny * G + nx) * COUT + kq;
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) {
      const bf16x4 a = *(const bf16x4*)(gp + ch * 16);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const bf16x4 bw = *(const bf16x4*)(wb + ((long long)(t * 16 + (lane & 15)) * 9 + tap) * COUT + ch * 16 + kq);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw, acc[t], 0, 0, 0);
      }
    }
  }
  const long long base = ((long long)b * G + row) * G * CIN;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int c = t * 16 + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = wv * 16 + (lane >> 4) * 4 + i;
      const long long q = base + (long long)p * CIN + c;
      gprev[q] = bf2f(xact[q]) > 0.f ? f2bf(acc[t][i]) : (uint16_t)0;
    }
  }
}

// Weight and bias gradients of one 3x3 layer, partial over kWgRows image rows
// of one image (blk = b (G / kWgRows) + row group):
//   part[blk][(o cin + c) 9 + tap] = sum_px X[px + off(tap)][c] G[px][o],
//   part[blk][cout cin 9 + o]      = sum_px G[px][o]   (real input channels only).
// For each tap the sum over pixels is a product with the pixels as the inner
// dimension, run on the 16x16x16 bf16 matrix cores: A = G^T (16 output
// channels x 16 pixels), B = X_tap (16 pixels x 16 input channels).  Per row
// the workgroup stages G^T [o][px] and, per tap, the shifted input row
// X_tap^T [c][px] in LDS, so that each lane's operand (4 consecutive pixels of
// one channel) is one 8-byte load.  Wave wv takes the (o, c) tile pair
// wv % PAIRS and the taps t with t % (4 / PAIRS) == wv / PAIRS.
template <int CINP, int COUT>
__global__ __launch_bounds__(256) void k_conv_bwd_w(const uint16_t* __restrict__ x, const uint16_t* __restrict__ g,
                                                    int cin, int dil, float* __restrict__ part) {
  constexpr int G = kNetGrid, GS = G + 4;  // LDS row stride (pixels), padded against bank conflicts
  constexpr int NO = COUT / 16, NCH = CINP / 16, PAIRS = NO * NCH, TSTEP = 4 / PAIRS;
  static_assert(PAIRS == 1 || PAIRS == 2 || PAIRS == 4, "tile pairs must divide the four waves");
  __shared__ __align__(16) uint16_t sgT[COUT][GS];
  __shared__ __align__(16) uint16_t sxT[9][CINP][GS];
  const int b = blockIdx.y, rg = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, kq = (lane >> 4) * 4;
  const int pair = wv % PAIRS, tsel = wv / PAIRS;
  const int o0 = (pair / NCH) * 16, c0 = (pair % NCH) * 16;
  floatx4 acc[9];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) acc[tap] = floatx4{0.f, 0.f, 0.f, 0.f};
  float bias = 0.f;  // thread o < COUT: sum of G[px][o] over the rows
  const uint16_t* xb = x + (long long)b * G * G * CINP;
  for (int rr = 0; rr < kWgRows; ++rr) {
    const int row = rg * kWgRows + rr;
    __syncthreads();  // the previous row's products are done with the LDS rows
    const uint16_t* gr = g + (((long long)b * G + row) * G) * COUT;
    for (int q = threadIdx.x; q < G * COUT; q += 256) sgT[q % COUT][q / COUT] = gr[q];
    for (int q = threadIdx.x; q < 9 * G * CINP; q += 256) {
      const int tap = q / (G * CINP), rem = q % (G * CINP), px = rem / CINP, c = rem % CINP;
      const int ny = (row + dil * (tap / 3 - 1) + 4 * G) % G;
      const int nx = (px + dil * (tap % 3 - 1) + 4 * G) % G;
      sxT[tap][c][px] = xb[((long long)ny * G + nx) * CINP + c];
    }
    __syncthreads();
    if (threadIdx.x < COUT)
      for (int px = 0; px < G; ++px) bias += bf2f(sgT[threadIdx.x][px]);
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      if (tap % TSTEP != tsel) continue;
#pragma unroll
      for (int k0 = 0; k0 < G; k0 += 16) {
        const bf16x4 av = *(const bf16x4*)&sgT[o0 + li][k0 + kq];
        const bf16x4 bv = *(const bf16x4*)&sxT[tap][c0 + li][k0 + kq];
        acc[tap] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[tap], 0, 0, 0);
      }
    }
  }
  // D[4 (lane / 16) + i][lane % 16] = dW_tap[o0 + kq + i][c0 + li]
  const int nw = COUT * cin * 9;
  float* out = part + ((long long)b * (G / kWgRows) + rg) * (nw + COUT);
  const int c = c0 + li;
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    if (tap % TSTEP != tsel || c >= cin) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) out[((long long)(o0 + kq + i) * cin + c) * 9 + tap] = acc[tap][i];
  }
  if (threadIdx.x < COUT) out[nw + threadIdx.x] = bias;
}

// grad[j] = sum_i part[i][j], j < count: a workgroup takes C adjacent columns
// (C = 16, 32 or 64, fewer for short gradients) and 256 / C interleaved row
// groups per column (rows i = grp, grp + 256 / C, ...), each summed in FP64,
// then added in group order (a fixed order for a given row count and C)
__global__ __launch_bounds__(256) void k_reduce_rows(const float* __restrict__ part, int rows, int count, int C,
                                                     float* __restrict__ grad) {
  __shared__ double sacc[256];
  const int NG = 256 / C;
  const int jl = threadIdx.x % C, grp = threadIdx.x / C;
  const int j = blockIdx.x * C + jl;
  double acc = 0.0;
  if (j < count)
    for (int i = grp; i < rows; i += NG) acc += part[(long long)i * count + j];
  sacc[threadIdx.x] = acc;
  __syncthreads();
  if (grp == 0 && j < count) {
    double tot = sacc[jl];
    for (int g = 1; g < NG; ++g) tot += sacc[g * C + jl];
    grad[j] = (float)tot;
  }
}

// --------------------------------------------------------------- the head
// o = w . h6 + b on the shifted grid; per pixel the loss terms
// d^2 G - 2 d H + Z with d = 1 / (k c), c = max(softplus(o), floor), and dL/do.
// k, G, H, Z are unshifted 64 x 64 maps of the training slice.
__global__ __launch_bounds__(256) void k_net_head(const uint16_t* __restrict__ h6, const float* __restrict__ theta,
                                                  int woff, const int* __restrict__ index, int batch,
                                                  const float* __restrict__ k, const float* __restrict__ Gs,
                                                  const float* __restrict__ Hs, const float* __restrict__ Zs,
                                                  const double* __restrict__ zsum, float* __restrict__ o_out,
                                                  float* __restrict__ go, double* __restrict__ loss_part) {
  constexpr int G = kNetGrid, CELLS = G * G;
  __shared__ double red[16];
  const int b = blockIdx.y, row = blockIdx.x;
  const int px = threadIdx.x;  // 64 threads per row
  const int cell = row * G + px;
  const uint16_t* hp = h6 + ((long long)b * CELLS + cell) * 16;
  float o = theta[woff + 16];
#pragma unroll
  for (int c = 0; c < 16; ++c) o += theta[woff + c] * bf2f(hp[c]);
  o_out[(long long)b * CELLS + cell] = o;
  double term = 0.0;
  if (k) {
    const int src = index ? index[b] : b;
    const int u = (row - G / 2 + G) % G, v = (px - G / 2 + G) % G;
    const long long q = (long long)src * CELLS + u * G + v;
    const float sp = softplus_f(o);
    const float c = fmaxf(sp, kNetFloor);
    const double d = 1.0 / ((double)k[q] * c);
    const double gq = Gs[q], hq = Hs[q], zq = Zs[q];
    const double zs = zsum[b];
    term = (d * d * gq - 2.0 * d * hq + zq) / zs;
    const double dLdd = (2.0 * d * gq - 2.0 * hq) / zs / batch;
    const double dcdo = sp > kNetFloor ? sigmoid_f(o) : 0.0;
    go[(long long)b * CELLS + cell] = (float)(dLdd * (-d / c) * dcdo);
  }
  term = block_sum_f64(term, red);
  if (threadIdx.x == 0) loss_part[(long long)b * G + row] = term;
}

// dL/d(pre-activation of layer 6) = go w (h6 > 0), plus the 1x1 layer's
// gradient partials: part[blk][c] = sum_px go h6[c], part[blk][16] = sum_px go.
__global__ __launch_bounds__(64) void k_net_head_bwd(const uint16_t* __restrict__ h6, const float* __restrict__ theta,
                                                     int woff, const float* __restrict__ go,
                                                     uint16_t* __restrict__ g6, float* __restrict__ part) {
  constexpr int G = kNetGrid, CELLS = G * G;
  __shared__ float sred[17][64];
  const int b = blockIdx.y, row = blockIdx.x, px = threadIdx.x;
  const int cell = row * G + px;
  const float gv = go[(long long)b * CELLS + cell];
  const uint16_t* hp = h6 + ((long long)b * CELLS + cell) * 16;
  uint16_t* gp = g6 + ((long long)b * CELLS + cell) * 16;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const float h = bf2f(hp[c]);
    gp[c] = h > 0.f ? f2bf(gv * theta[woff + c]) : (uint16_t)0;
    sred[c][px] = gv * h;
  }
  sred[16][px] = gv;
  __syncthreads();
  if (px < 17) {
    float acc = 0.f;
    for (int i = 0; i < 64; ++i) acc += sred[px][i];
    part[((long long)b * G + row) * 17 + px] = acc;
  }
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ theta, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int count, float lr,
                                              float c1, float c2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// correction for every slice of a context: c = max(softplus(o), floor) on the
// shifted 64 x 64 grid, periodic bilinear interpolation to m x n (shifted,
// cell-centred), written back in unshifted order.
__global__ __launch_bounds__(256) void k_net_upsample(Ws w, const float* __restrict__ o, int slice0,
                                                      float* __restrict__ corr) {
  constexpr int G = kNetGrid;
  const int s = slice0 + blockIdx.y;
  const SliceDev sd = w.sl[s];
  const int m = sd.m, n = sd.n;
  const float* ob = o + (long long)blockIdx.y * G * G;
  const long long np = (long long)m * n;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < np; p += (long long)gridDim.x * blockDim.x) {
    const int ps = int(p / n), qs = int(p % n);  // shifted position
    const float fy = (ps + 0.5f) / (m / G) - 0.5f, fx = (qs + 0.5f) / (n / G) - 0.5f;
    const int y0 = (int)floorf(fy), x0 = (int)floorf(fx);
    const float ty = fy - y0, tx = fx - x0;
    const int ya = (y0 + G) % G, yb = (y0 + 1 + G) % G, xa = (x0 + G) % G, xb = (x0 + 1 + G) % G;
    auto cval = [&](int yy, int xx) { return fmaxf(softplus_f(ob[yy * G + xx]), kNetFloor); };
    const float v = (1.f - ty) * ((1.f - tx) * cval(ya, xa) + tx * cval(ya, xb)) +
                    ty * ((1.f - tx) * cval(yb, xa) + tx * cval(yb, xb));
    const int u = (ps - m / 2 + m) % m, vv = (qs - n / 2 + n) % n;
    corr[sd.img + (long long)u * n + vv] = v;
  }
}

// probe statistics accumulation, unitary scaling 1/N folded in
__global__ __launch_bounds__(256) void k_probe_accum(Ws w, const float2* __restrict__ fa, const float2* __restrict__ fz,
                                                     float* __restrict__ G, float* __restrict__ H,
                                                     float* __restrict__ Z, float weight, int first) {
  const int s = blockIdx.y;
  const SliceDev sd = w.sl[s];
  const long long np = (long long)sd.m * sd.n;
  const float sc = weight / (float)np;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < np; p += (long long)gridDim.x * blockDim.x) {
    const long long q = sd.img + p;
    const float2 a = fa[q], z = fz[q];
    const float g = sc * (a.x * a.x + a.y * a.y), h = sc * (a.x * z.x + a.y * z.y), zz = sc * (z.x * z.x + z.y * z.y);
    G[q] = first ? g : G[q] + g;
    H[q] = first ? h : H[q] + h;
    Z[q] = first ? zz : Z[q] + zz;
  }
}

// out[b] = sum of the 64 x 64 plane of slice index[b] (FP64)
__global__ __launch_bounds__(256) void k_plane_sums(const float* __restrict__ z, const int* __restrict__ index,
                                                    double* __restrict__ out) {
  __shared__ double red[16];
  constexpr int CELLS = kNetGrid * kNetGrid;
  const long long src = index ? index[blockIdx.x] : blockIdx.x;
  double a = 0.0;
  for (int c = threadIdx.x; c < CELLS; c += blockDim.x) a += z[src * CELLS + c];
  a = block_sum_f64(a, red);
  if (threadIdx.x == 0) out[blockIdx.x] = a;
}

// ============================================================== launchers

hipError_t launch_features(hipStream_t st, const Ws& w, int nslices, const float* energy, const float* kraw,
                           float* feat) {
  hipLaunchKernelGGL(k_features, dim3(nslices), dim3(256), 0, st, w, energy, kraw, feat);
  return hipGetLastError();
}

hipError_t launch_net_prep(hipStream_t st, const float* theta, const NetLayout& L) {
  hipLaunchKernelGGL(k_net_prep, dim3(16, kNetLayers), dim3(256), 0, st, theta, L);
  return hipGetLastError();
}

hipError_t launch_net_input(hipStream_t st, const float* feat, const int* index, int batch, uint16_t* x0) {
  hipLaunchKernelGGL(k_net_input, dim3(64, batch), dim3(256), 0, st, feat, index, x0);
  return hipGetLastError();
}

hipError_t launch_conv_fwd(hipStream_t st, int cinp, int cout, const uint16_t* x, const uint16_t* wf,
                           const float* bias, int dil, int batch, uint16_t* y) {
  const dim3 grid(kNetGrid, batch);
  if (cinp == 16 && cout == 32) hipLaunchKernelGGL((k_conv_fwd<16, 32>), grid, dim3(256), 0, st, x, wf, bias, dil, y);
  else if (cinp == 32 && cout == 32) hipLaunchKernelGGL((k_conv_fwd<32, 32>), grid, dim3(256), 0, st, x, wf, bias, dil, y);
  else if (cinp == 32 && cout == 16) hipLaunchKernelGGL((k_conv_fwd<32, 16>), grid, dim3(256), 0, st, x, wf, bias, dil, y);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_conv_bwd_data(hipStream_t st, int cinp, int cout, const uint16_t* g, const uint16_t* wb,
                                const uint16_t* xact, int dil, int batch, uint16_t* gprev) {
  const dim3 grid(kNetGrid, batch);
  if (cinp == 32 && cout == 32)
    hipLaunchKernelGGL((k_conv_bwd_data<32, 32>), grid, dim3(256), 0, st, g, wb, xact, dil, gprev);
  else if (cinp == 32 && cout == 16)
    hipLaunchKernelGGL((k_conv_bwd_data<32, 16>), grid, dim3(256), 0, st, g, wb, xact, dil, gprev);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_conv_bwd_w(hipStream_t st, int cinp, int cin, int cout, const uint16_t* x, const uint16_t* g,
                             int dil, int batch, float* part) {
  const dim3 grid(kNetGrid / kWgRows, batch);
  if (cinp == 16 && cout == 32) hipLaunchKernelGGL((k_conv_bwd_w<16, 32>), grid, dim3(256), 0, st, x, g, cin, dil, part);
  else if (cinp == 32 && cout == 32)
    hipLaunchKernelGGL((k_conv_bwd_w<32, 32>), grid, dim3(256), 0, st, x, g, cin, dil, part);
  else if (cinp == 32 && cout == 16)
    hipLaunchKernelGGL((k_conv_bwd_w<32, 16>), grid, dim3(256), 0, st, x, g, cin, dil, part);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_reduce_rows(hipStream_t st, const float* part, int rows, int count, float* grad) {
  const int C = count >= 64 ? 64 : count >= 32 ? 32 : 16;
  hipLaunchKernelGGL(k_reduce_rows, dim3((count + C - 1) / C), dim3(256), 0, st, part, rows, count, C, grad);
  return hipGetLastError();
}

hipError_t launch_net_head(hipStream_t st, const uint16_t* h6, const float* theta, int woff, const int* index,
                           int batch, const float* k, const float* G, const float* H, const float* Z,
                           const double* zsum, float* o, float* go, double* loss_part) {
  hipLaunchKernelGGL(k_net_head, dim3(kNetGrid, batch), dim3(64), 0, st, h6, theta, woff, index, batch, k, G, H, Z,
                     zsum, o, go, loss_part);
  return hipGetLastError();
}

hipError_t launch_net_head_bwd(hipStream_t st, const uint16_t* h6, const float* theta, int woff, const float* go,
                               int batch, uint16_t* g6, float* part) {
  hipLaunchKernelGGL(k_net_head_bwd, dim3(kNetGrid, batch), dim3(64), 0, st, h6, theta, woff, go, g6, part);
  return hipGetLastError();
}

hipError_t launch_adam(hipStream_t st, float* theta, const float* g, float* m, float* v, int count, float lr, int t) {
  const float c1 = 1.f - powf(0.9f, (float)t), c2 = 1.f - powf(0.999f, (float)t);
  hipLaunchKernelGGL(k_adam, dim3(std::max(1, std::min(256, (count + 255) / 256))), dim3(256), 0, st, theta, g, m, v,
                     count, lr, c1, c2);
  return hipGetLastError();
}

hipError_t launch_net_upsample(hipStream_t st, const Ws& w, const float* o, int slice0, int count,
                               long long max_pixels, float* corr) {
  long long blocks = (max_pixels + 255) / 256;
  blocks = std::min(blocks, 1024LL);
  hipLaunchKernelGGL(k_net_upsample, dim3((unsigned)blocks, count), dim3(256), 0, st, w, o, slice0, corr);
  return hipGetLastError();
}

hipError_t launch_probe_accum(const Simple& S, const Ws& w, const float2* fa, const float2* fz, float* G, float* H,
                              float* Z, float weight, int first) {
  long long blocks = std::min((S.max_pixels + 255) / 256, 1024LL);
  hipLaunchKernelGGL(k_probe_accum, dim3((unsigned)blocks, S.nslices), dim3(256), 0, S.stream, w, fa, fz, G, H, Z,
                     weight, first);
  return hipGetLastError();
}

hipError_t launch_plane_sums_indexed(hipStream_t st, const float* z, const int* index, int count, double* out) {
  hipLaunchKernelGGL(k_plane_sums, dim3(count), dim3(256), 0, st, z, index, out);
  return hipGetLastError();
}

}  // namespace pics

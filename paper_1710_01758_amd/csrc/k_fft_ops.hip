// FFT-based kernels: the fused line-mask system operator, the circulant
// preconditioner passes, the PCG vector updates and the FFT passes used by
// Split Bregman's initialisation and the preconditioner build.
//
// Column tiles: a workgroup owns T = 16 adjacent columns of one slice and all
// m rows; thread (t, j) holds rows t + NT e of column j (cyclic layout), so a
// length-m transform along axis 0 runs in registers + LDS.  Row tiles: a
// workgroup owns 16 rows, thread (t, r) holds columns t + NT e of row r.
#include "fft.hpp"
#include "internal.hpp"

namespace pics {

template <int M>
struct ColCfg {
  static constexpr int NT = Plan<M>::NT;
  static constexpr int E = M / NT;
  static constexpr int T = kColT;
  static constexpr int THREADS = NT * T;
};
template <int N>
struct RowCfg {
  static constexpr int NT = Plan<N>::NT;
  static constexpr int E = N / NT;
  static constexpr int RR = kRowRR;
  static constexpr int THREADS = NT * RR;
  static constexpr int LDS = RR * RowLay<N>::stride;
};

// Stop rule shared by every kernel that tests convergence: relative residual
// ||r|| <= tol ||b|| (recursive residual), or the per-slice iteration cap.
__device__ __forceinline__ bool pcg_should_stop(const Ws& w, int s, int m, double tol, int* status) {
  const PcgState* st = w.st + s;
  const int nrt = m / kRowRR;
  const double rr = part_sum(part_ptr(w.part, s, P_RR), nrt);
  const double bb = part_sum(part_ptr(w.part, s, P_BB), nrt);
  if (rr <= tol * tol * bb) {
    *status = 1;
    return true;
  }
  if (st->it_a >= st->maxit) {
    *status = 0;
    return true;
  }
  return false;
}

__device__ __forceinline__ void pcg_mark_done(const Ws& w, int s, int status, double tol) {
  PcgState* st = w.st + s;
  const SliceDev& sd = w.sl[s];
  const int nrt = sd.m / kRowRR;
  const double rr = part_sum(part_ptr(w.part, s, P_RR), nrt);
  const double bb = part_sum(part_ptr(w.part, s, P_BB), nrt);
  st->done = 1;
  st->status = status;
  st->iters = st->it_a;
  st->relres = bb > 0.0 ? sqrt(rr / bb) : 0.0;
}

// ----------------------------------------------------------------------------
// System operator with a line mask, one column tile per workgroup:
//   out = mu sum_c conj(S_c) F_m^H diag(r) F_m (S_c p) + lam (D_x^H D_x + D_y^H D_y) p + gam p
// (Eq. system with W^H W = I).  A line mask samples whole k-space rows, so
// F^H R F factors into a length-m transform along axis 0 only; the 1/m of the
// unitary pair is folded into the mask.
// Modes: CA_APPLY  p = xin
//        CA_PCG    p = zs + beta p_old (beta from the rho partials), written to pn;
//                  sigma = Re(p^H A p) partial
//        CA_OUTER  p = xin; also g <- g + g1 - (data term)
// ----------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(ColCfg<M>::THREADS) void k_col_apply(
    Ws w, int mode, int terms, int pk, double tol, const float2* __restrict__ xin, const float2* __restrict__ zsrc,
    const float2* __restrict__ pold, float2* __restrict__ pn, float2* __restrict__ out, float2* __restrict__ g,
    const float2* __restrict__ g1) {
  constexpr int NT = ColCfg<M>::NT, E = ColCfg<M>::E, T = kColT, TH = ColCfg<M>::THREADS;
  constexpr int TS = T + 2;  // tile stride with the two halo columns
  __shared__ float2 lds[M * TS];
  __shared__ double red[16];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  const int n = sd.n;
  const int j = threadIdx.x % T, t = threadIdx.x / T;
  const int j0 = blockIdx.x * T;
  const int col = j0 + j;
  const long long base = sd.img;

  int it = 0;
  float beta = 0.f;
  bool first = true;
  if (mode == CA_PCG) {
    PcgState* st = w.st + s;
    if (st->done) return;
    int status;
    if (pcg_should_stop(w, s, sd.m, tol, &status)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) pcg_mark_done(w, s, status, tol);
      return;
    }
    it = st->it_a;
    first = (it == 0);
    if (!first) {
      const int nrt = sd.m / kRowRR;
      const double rho_i = part_sum(part_ptr(w.part, s, P_RHO0 + (it & 1)), nrt);
      const double rho_p = part_sum(part_ptr(w.part, s, P_RHO0 + ((it - 1) & 1)), nrt);
      beta = float(rho_i / rho_p);
    }
  }

  auto pval = [&](long long idx) -> float2 {
    if (mode != CA_PCG) return xin[idx];
    float2 zs;
    if (pk == PK_NONE) {
      zs = zsrc[idx];
    } else if (pk == PK_JACOBI) {
      zs = cscale(zsrc[idx], w.jac[idx]);
    } else {
      zs = zsrc[idx];
    }
    if (first) return zs;
    const float2 po = pold[idx];
    return make_float2(zs.x + beta * po.x, zs.y + beta * po.y);
  };

  float2 pv[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = t + NT * e;
    const long long idx = base + (long long)i * n + col;
    pv[e] = pval(idx);
    lds[i * TS + j + 1] = pv[e];
    if (mode == CA_PCG) pn[idx] = pv[e];
  }
  const int jl = (j0 - 1 + n) % n, jr = (j0 + T) % n;
  for (int h = threadIdx.x; h < 2 * M; h += TH) {
    const int side = h / M, i = h % M;
    const int jh = side ? jr : jl;
    lds[i * TS + (side ? T + 1 : 0)] = pval(base + (long long)i * n + jh);
  }
  __syncthreads();
  // q starts as the diagonal-in-Fourier terms lam (D_x^H D_x + D_y^H D_y) p + gam p
  float2 q[E];
  const float mu = sd.mu, lam = sd.lam, gam = sd.gam;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = t + NT * e;
    float2 a = make_float2(0.f, 0.f);
    if (terms & TERM_TV) {
      const int iu = (i - 1 + M) % M, id = (i + 1) % M;
      const float2 c = lds[i * TS + j + 1];
      const float2 u = lds[iu * TS + j + 1], d = lds[id * TS + j + 1];
      const float2 l = lds[i * TS + j], r = lds[i * TS + j + 2];
      a = make_float2(lam * (4.f * c.x - u.x - d.x - l.x - r.x), lam * (4.f * c.y - u.y - d.y - l.y - r.y));
    }
    if (terms & TERM_GAMMA) a = make_float2(a.x + gam * pv[e].x, a.y + gam * pv[e].y);
    q[e] = a;
  }
  __syncthreads();

  // data term, accumulated coil by coil: mu conj(S_c) F^H R F (S_c p)
  float2 dat[E];
#pragma unroll
  for (int e = 0; e < E; ++e) dat[e] = make_float2(0.f, 0.f);
  if (terms & TERM_DATA) {
    const uint8_t* mk = w.mask + sd.mask;
    unsigned mbits = 0u;  // bit e: frequency row t + NT e sampled
#pragma unroll
    for (int e = 0; e < E; ++e) mbits |= (mk[t + NT * e] ? 1u : 0u) << e;
    const float inv_m = 1.0f / M;
    const float2* __restrict__ tw = w.tw + tw_offset(M);
    const float2* S = w.sens + sd.coil;
    for (int c = 0; c < sd.nc; ++c) {
      const float2* Sc = S + (long long)c * M * n;
      float2 sv[E], v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int i = t + NT * e;
        sv[e] = Sc[(long long)i * n + col];
        v[e] = cmul(sv[e], pv[e]);
      }
      fft<M, -1, ColLay<T>>(v, t, lds, j, tw);
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = cscale(v[e], ((mbits >> e) & 1u) ? inv_m : 0.f);
      fft<M, +1, ColLay<T>>(v, t, lds, j, tw);
#pragma unroll
      for (int e = 0; e < E; ++e) dat[e] = cadd(dat[e], cconjmul(sv[e], v[e]));
    }
  }

  double sig = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = t + NT * e;
    const long long idx = base + (long long)i * n + col;
    const float2 qv = make_float2(q[e].x + mu * dat[e].x, q[e].y + mu * dat[e].y);
    out[idx] = qv;
    sig += (double)pv[e].x * (double)qv.x + (double)pv[e].y * (double)qv.y;
    if (mode == CA_OUTER) {
      const float2 gv = g[idx], g1v = g1[idx];
      g[idx] = make_float2(gv.x + g1v.x - mu * dat[e].x, gv.y + g1v.y - mu * dat[e].y);
    }
  }
  if (mode == CA_PCG) {
    sig = block_sum_f64(sig, red);
    if (threadIdx.x == 0) {
      part_ptr(w.part, s, P_SIGMA)[blockIdx.x] = sig;
      if (blockIdx.x == 0) w.st[s].it_r = it;
    }
  }
}

// ----------------------------------------------------------------------------
// PCG vector update + residual norm, then the first pass of M^{-1} r (row
// FFTs), one row tile per workgroup.
//   RU_SETUP : r = b - q (q = A x0); ||b||^2 and ||r||^2 partials
//   RU_UPDATE: alpha = rho / sigma; x += alpha pn; r -= alpha q; p = pn
// Circulant / learned: t = row-FFT(r).  None / Jacobi: rho' = Re(r^H z)
// partial with z = r or z = r / diag(A).
// ----------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void k_row_update(Ws w, int mode, int pk,
                                                                   const float2* __restrict__ b,
                                                                   const float2* __restrict__ q, float2* x, float2* r,
                                                                   const float2* __restrict__ pn, float2* p,
                                                                   float2* __restrict__ tout) {
  constexpr int NT = RowCfg<N>::NT, E = RowCfg<N>::E;
  __shared__ float2 lds[RowCfg<N>::LDS];
  __shared__ double red[16];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  PcgState* st = w.st + s;
  const int t = threadIdx.x % NT, rr_ = threadIdx.x / NT;
  const int i = blockIdx.x * kRowRR + rr_;
  const long long rowbase = sd.img + (long long)i * N;

  int it = 0;
  float alpha = 0.f;
  if (mode == RU_UPDATE) {
    if (st->done) return;
    it = st->it_r;
    const int nrt = sd.m / kRowRR, nct = N / kColT;
    const double sigma = part_sum(part_ptr(w.part, s, P_SIGMA), nct);
    const double rho = part_sum(part_ptr(w.part, s, P_RHO0 + (it & 1)), nrt);
    const double a = rho / sigma;
    if (!(sigma > 0.0) || !isfinite(a)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->done = 1;
        st->status = isfinite(sigma) && isfinite(rho) ? -4 : -3;
        st->iters = it;
      }
      return;
    }
    alpha = float(a);
  }

  float2 v[E];
  double rrp = 0.0, bbp = 0.0, rhop = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const long long idx = rowbase + t + NT * e;
    float2 rv;
    if (mode == RU_UPDATE) {
      const float2 pnv = pn[idx];
      const float2 xv = x[idx];
      x[idx] = make_float2(xv.x + alpha * pnv.x, xv.y + alpha * pnv.y);
      const float2 ro = r[idx], qv = q[idx];
      rv = make_float2(ro.x - alpha * qv.x, ro.y - alpha * qv.y);
      p[idx] = pnv;
    } else {
      const float2 bv = b[idx], qv = q[idx];
      rv = csub(bv, qv);
      bbp += (double)bv.x * bv.x + (double)bv.y * bv.y;
    }
    r[idx] = rv;
    const double a2 = (double)rv.x * rv.x + (double)rv.y * rv.y;
    rrp += a2;
    if (pk == PK_JACOBI) rhop += (double)w.jac[idx] * a2;
    if (pk == PK_NONE) rhop += a2;
    v[e] = rv;
  }
  rrp = block_sum_f64(rrp, red);
  if (threadIdx.x == 0) part_ptr(w.part, s, P_RR)[blockIdx.x] = rrp;
  if (mode == RU_SETUP) {
    bbp = block_sum_f64(bbp, red);
    if (threadIdx.x == 0) part_ptr(w.part, s, P_BB)[blockIdx.x] = bbp;
  }
  const int rho_slot = P_RHO0 + ((mode == RU_SETUP) ? 0 : ((it + 1) & 1));
  if (pk == PK_NONE || pk == PK_JACOBI) {
    rhop = block_sum_f64(rhop, red);
    if (threadIdx.x == 0) part_ptr(w.part, s, rho_slot)[blockIdx.x] = rhop;
  } else {
    const float2* __restrict__ tw = w.tw + tw_offset(N);
    fft<N, -1, RowLay<N>>(v, t, lds, rr_, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) tout[rowbase + t + NT * e] = v[e];
  }
  if (mode == RU_UPDATE && blockIdx.x == 0 && threadIdx.x == 0) st->it_a = it + 1;
}

// ----------------------------------------------------------------------------
// Middle pass of M^{-1} = F^H diag(1/k) F: column FFT, scale by 1/(k m n),
// inverse column FFT, in place.  With `check` the stop rule is tested first.
// use_state = 0 ignores the PCG control block (stand-alone M^{-1}).
// ----------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(ColCfg<M>::THREADS) void k_col_precond(Ws w, int use_state, int check, double tol,
                                                                     float2* __restrict__ tbuf) {
  constexpr int NT = ColCfg<M>::NT, E = ColCfg<M>::E, T = kColT;
  __shared__ float2 lds[M * T];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  if (use_state) {
    if (w.st[s].done) return;
    int status;
    if (check && pcg_should_stop(w, s, sd.m, tol, &status)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) pcg_mark_done(w, s, status, tol);
      return;
    }
  }
  const int n = sd.n;
  const int j = threadIdx.x % T, t = threadIdx.x / T;
  const int col = blockIdx.x * T + j;
  const long long base = sd.img;
  const float2* __restrict__ tw = w.tw + tw_offset(M);
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = tbuf[base + (long long)(t + NT * e) * n + col];
  fft<M, -1, ColLay<T>>(v, t, lds, j, tw);
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = cscale(v[e], w.kinv[base + (long long)(t + NT * e) * n + col]);
  fft<M, +1, ColLay<T>>(v, t, lds, j, tw);
#pragma unroll
  for (int e = 0; e < E; ++e) tbuf[base + (long long)(t + NT * e) * n + col] = v[e];
}

// ----------------------------------------------------------------------------
// Last pass of M^{-1}: inverse row FFT -> z, and rho = Re(r^H z) partial.
// ----------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void k_row_z(Ws w, const float2* __restrict__ tbuf,
                                                              const float2* __restrict__ r, float2* __restrict__ z) {
  constexpr int NT = RowCfg<N>::NT, E = RowCfg<N>::E;
  __shared__ float2 lds[RowCfg<N>::LDS];
  __shared__ double red[16];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  PcgState* st = w.st + s;
  if (st->done) return;
  const int t = threadIdx.x % NT, rr_ = threadIdx.x / NT;
  const int i = blockIdx.x * kRowRR + rr_;
  const long long rowbase = sd.img + (long long)i * N;
  const float2* __restrict__ tw = w.tw + tw_offset(N);
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = tbuf[rowbase + t + NT * e];
  fft<N, +1, RowLay<N>>(v, t, lds, rr_, tw);
  double rho = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const long long idx = rowbase + t + NT * e;
    z[idx] = v[e];
    const float2 rv = r[idx];
    rho += (double)rv.x * v[e].x + (double)rv.y * v[e].y;
  }
  rho = block_sum_f64(rho, red);
  if (threadIdx.x == 0) part_ptr(w.part, s, P_RHO0 + (st->it_a & 1))[blockIdx.x] = rho;
}

// ----------------------------------------------------------------------------
// Plain row FFT (unnormalised).  ncoil_mode: loop over the slice's coils on
// coil-shaped buffers, zeroing unsampled k-space first (R y before F^H).
// ----------------------------------------------------------------------------
template <int N, int DIR>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void k_row_fft(Ws w, int ncoil_mode, const float2* __restrict__ in,
                                                                float2* __restrict__ out) {
  constexpr int NT = RowCfg<N>::NT, E = RowCfg<N>::E;
  __shared__ float2 lds[RowCfg<N>::LDS];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  const int t = threadIdx.x % NT, rr_ = threadIdx.x / NT;
  const int i = blockIdx.x * kRowRR + rr_;
  const float2* __restrict__ tw = w.tw + tw_offset(N);
  const int ncoil = ncoil_mode ? sd.nc : 1;
  const long long plane = (long long)sd.m * N;
  const uint8_t* mk = w.mask + sd.mask;
  for (int c = 0; c < ncoil; ++c) {
    const long long rowbase = (ncoil_mode ? sd.coil + c * plane : sd.img) + (long long)i * N;
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      float2 a = in[rowbase + t + NT * e];
      if (ncoil_mode) {
        const bool keep = sd.mask_kind == 0 ? mk[i] != 0 : mk[(long long)i * N + t + NT * e] != 0;
        if (!keep) a = make_float2(0.f, 0.f);
      }
      v[e] = a;
    }
    fft<N, DIR, RowLay<N>>(v, t, lds, rr_, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) out[rowbase + t + NT * e] = v[e];
  }
}

// Plain column FFT (unnormalised), image-shaped buffers.
template <int M, int DIR>
__global__ __launch_bounds__(ColCfg<M>::THREADS) void k_col_fft(Ws w, const float2* __restrict__ in,
                                                                float2* __restrict__ out) {
  constexpr int NT = ColCfg<M>::NT, E = ColCfg<M>::E, T = kColT;
  __shared__ float2 lds[M * T];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  const int n = sd.n;
  const int j = threadIdx.x % T, t = threadIdx.x / T;
  const int col = blockIdx.x * T + j;
  const float2* __restrict__ tw = w.tw + tw_offset(M);
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = in[sd.img + (long long)(t + NT * e) * n + col];
  fft<M, DIR, ColLay<T>>(v, t, lds, j, tw);
#pragma unroll
  for (int e = 0; e < E; ++e) out[sd.img + (long long)(t + NT * e) * n + col] = v[e];
}

// ----------------------------------------------------------------------------
// Split Bregman initialisation (Algorithm 1, step 1 and the data part of the
// first right-hand side): per coil, finish the 2D inverse FFT of R y_c along
// axis 0 (the row pass already ran), scale to the unitary F^H, and form
//   g1 = mu sum_c conj(S_c) m_c,   x = sqrt(sum_c |m_c|^2)   (root sum of squares)
// ----------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(ColCfg<M>::THREADS) void k_col_sb_init(Ws w, const float2* __restrict__ coil_rows,
                                                                     float2* __restrict__ g1, float2* __restrict__ g,
                                                                     float2* __restrict__ x) {
  constexpr int NT = ColCfg<M>::NT, E = ColCfg<M>::E, T = kColT;
  __shared__ float2 lds[M * T];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  const int n = sd.n;
  const int j = threadIdx.x % T, t = threadIdx.x / T;
  const int col = blockIdx.x * T + j;
  const float2* __restrict__ tw = w.tw + tw_offset(M);
  const float scale = 1.0f / sqrtf((float)M * (float)n);
  float2 acc[E];
  float sos[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    acc[e] = make_float2(0.f, 0.f);
    sos[e] = 0.f;
  }
  for (int c = 0; c < sd.nc; ++c) {
    const long long cb = sd.coil + (long long)c * M * n;
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = coil_rows[cb + (long long)(t + NT * e) * n + col];
    fft<M, +1, ColLay<T>>(v, t, lds, j, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const float2 mc = cscale(v[e], scale);
      const float2 sv = w.sens[cb + (long long)(t + NT * e) * n + col];
      acc[e] = cadd(acc[e], cconjmul(sv, mc));
      sos[e] += cabs2(mc);
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const long long idx = sd.img + (long long)(t + NT * e) * n + col;
    const float2 gv = cscale(acc[e], sd.mu);
    g1[idx] = gv;
    g[idx] = gv;
    x[idx] = make_float2(sqrtf(sos[e]), 0.f);
  }
}

// ----------------------------------------------------------------------------
// Preconditioner build, line masks.  With r constant along axis 1,
// k_c(u) = (1/N^2) sum_l r(l) Pbar(l - u), Pbar(t) = sum_v P(t, v), and by
// Parseval along axis 1, Pbar(t) = n sum_c sum_col |DFT_m(s_c[:, col])(t)|^2:
// only the axis-0 transforms of the coil maps are needed.  This kernel writes
// one partial Pbar per column tile (FP64) and the per-pixel coil energy
// sum_c |S_c|^2 (for the Jacobi diagonal) into `jac`.
// ----------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(ColCfg<M>::THREADS) void k_col_coil_power(Ws w, double* __restrict__ pbar,
                                                                        float* __restrict__ energy) {
  constexpr int NT = ColCfg<M>::NT, E = ColCfg<M>::E, T = kColT;
  __shared__ float2 lds[M * T];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  const int n = sd.n;
  const int j = threadIdx.x % T, t = threadIdx.x / T;
  const int col = blockIdx.x * T + j;
  const float2* __restrict__ tw = w.tw + tw_offset(M);
  double pw[E];
  float en[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    pw[e] = 0.0;
    en[e] = 0.f;
  }
  for (int c = 0; c < sd.nc; ++c) {
    const long long cb = sd.coil + (long long)c * M * n;
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      v[e] = w.sens[cb + (long long)(t + NT * e) * n + col];
      en[e] += cabs2(v[e]);
    }
    fft<M, -1, ColLay<T>>(v, t, lds, j, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) pw[e] += (double)v[e].x * v[e].x + (double)v[e].y * v[e].y;
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    energy[sd.img + (long long)(t + NT * e) * n + col] = en[e];
    double a = pw[e];
    // sum over the T columns of the tile: lanes j = 0..T-1 are adjacent
#pragma unroll
    for (int off = T / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if (j == 0) pbar[sd.aux + (long long)blockIdx.x * M + (t + NT * e)] = a;
  }
}

// ============================================================== launchers

#define PICS_FFT_SIZES(X) X(64) X(128) X(192) X(224) X(256) X(320) X(512)

hipError_t launch_col_apply(const Launch& L, const Ws& w, int mode, int terms, int pk, double tol,
                            const float2* xin, const float2* zsrc, const float2* pold, float2* pn, float2* out,
                            float2* g, const float2* g1) {
  const dim3 grid(L.n / kColT, L.count);
  switch (L.m) {
#define PICS_CASE(M)                                                                                          \
  case M:                                                                                                     \
    hipLaunchKernelGGL(k_col_apply<M>, grid, dim3(ColCfg<M>::THREADS), 0, L.stream, w, mode, terms, pk, tol, \
                       xin, zsrc, pold, pn, out, g, g1);                                                      \
    break;
    PICS_FFT_SIZES(PICS_CASE)
#undef PICS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_row_update(const Launch& L, const Ws& w, int mode, int pk, const float2* b, const float2* q,
                             float2* x, float2* r, const float2* pn, float2* p, float2* t) {
  const dim3 grid(L.m / kRowRR, L.count);
  switch (L.n) {
#define PICS_CASE(N)                                                                                      \
  case N:                                                                                                 \
    hipLaunchKernelGGL(k_row_update<N>, grid, dim3(RowCfg<N>::THREADS), 0, L.stream, w, mode, pk, b, q, x, \
                       r, pn, p, t);                                                                      \
    break;
    PICS_FFT_SIZES(PICS_CASE)
#undef PICS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_col_precond(const Launch& L, const Ws& w, int use_state, int check, double tol, float2* t) {
  const dim3 grid(L.n / kColT, L.count);
  switch (L.m) {
#define PICS_CASE(M)                                                                                           \
  case M:                                                                                                      \
    hipLaunchKernelGGL(k_col_precond<M>, grid, dim3(ColCfg<M>::THREADS), 0, L.stream, w, use_state, check, tol, \
                       t);                                                                                     \
    break;
    PICS_FFT_SIZES(PICS_CASE)
#undef PICS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_row_z(const Launch& L, const Ws& w, const float2* t, const float2* r, float2* z) {
  const dim3 grid(L.m / kRowRR, L.count);
  switch (L.n) {
#define PICS_CASE(N)                                                                             \
  case N:                                                                                        \
    hipLaunchKernelGGL(k_row_z<N>, grid, dim3(RowCfg<N>::THREADS), 0, L.stream, w, t, r, z); \
    break;
    PICS_FFT_SIZES(PICS_CASE)
#undef PICS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_row_fft(const Launch& L, const Ws& w, int inverse, int ncoil_mode, const float2* in, float2* out) {
  const dim3 grid(L.m / kRowRR, L.count);
  switch (L.n) {
#define PICS_CASE(N)                                                                                      \
  case N:                                                                                                 \
    if (inverse)                                                                                          \
      hipLaunchKernelGGL((k_row_fft<N, 1>), grid, dim3(RowCfg<N>::THREADS), 0, L.stream, w, ncoil_mode, in, \
                         out);                                                                            \
    else                                                                                                  \
      hipLaunchKernelGGL((k_row_fft<N, -1>), grid, dim3(RowCfg<N>::THREADS), 0, L.stream, w, ncoil_mode, in, \
                         out);                                                                            \
    break;
    PICS_FFT_SIZES(PICS_CASE)
#undef PICS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_col_fft(const Launch& L, const Ws& w, int inverse, const float2* in, float2* out) {
  const dim3 grid(L.n / kColT, L.count);
  switch (L.m) {
#define PICS_CASE(M)                                                                                          \
  case M:                                                                                                     \
    if (inverse)                                                                                              \
      hipLaunchKernelGGL((k_col_fft<M, 1>), grid, dim3(ColCfg<M>::THREADS), 0, L.stream, w, in, out);        \
    else                                                                                                      \
      hipLaunchKernelGGL((k_col_fft<M, -1>), grid, dim3(ColCfg<M>::THREADS), 0, L.stream, w, in, out);       \
    break;
    PICS_FFT_SIZES(PICS_CASE)
#undef PICS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_col_sb_init(const Launch& L, const Ws& w, const float2* coil_rows, float2* g1, float2* g,
                              float2* x) {
  const dim3 grid(L.n / kColT, L.count);
  switch (L.m) {
#define PICS_CASE(M)                                                                                             \
  case M:                                                                                                        \
    hipLaunchKernelGGL(k_col_sb_init<M>, grid, dim3(ColCfg<M>::THREADS), 0, L.stream, w, coil_rows, g1, g, x); \
    break;
    PICS_FFT_SIZES(PICS_CASE)
#undef PICS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_col_coil_power(const Launch& L, const Ws& w, double* pbar, float* energy) {
  const dim3 grid(L.n / kColT, L.count);
  switch (L.m) {
#define PICS_CASE(M)                                                                                           \
  case M:                                                                                                      \
    hipLaunchKernelGGL(k_col_coil_power<M>, grid, dim3(ColCfg<M>::THREADS), 0, L.stream, w, pbar, energy); \
    break;
    PICS_FFT_SIZES(PICS_CASE)
#undef PICS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool fft_size_supported(int N) {
  switch (N) {
#define PICS_CASE(X) case X:
    PICS_FFT_SIZES(PICS_CASE)
#undef PICS_CASE
    return true;
    default:
      return false;
  }
}

}  // namespace pics

// FFT-based kernels: the fused line-mask system operator, the circulant
// preconditioner passes, the PCG vector updates and the FFT passes used by
// Split Bregman's initialisation and the preconditioner build.
//
// Column tiles: a workgroup owns T = 16 adjacent columns of one slice and all
// m rows; thread (t, j) holds rows t + NT e of column j (cyclic layout), so a
// length-m transform along axis 0 runs in registers + LDS.  Row tiles: a
// workgroup owns 16 rows, thread (t, r) holds columns t + NT e of row r.
#include <type_traits>

#include "tiles.hpp"

namespace pics {

// ----------------------------------------------------------------------------
// System operator with a line mask, one column tile per workgroup:
//   out = mu sum_c conj(S_c) F_m^H diag(r) F_m (S_c p) + lam (D_x^H D_x + D_y^H D_y) p + gam p
// (Eq. system with W^H W = I).  A line mask samples whole k-space rows, so
// F^H R F factors into a length-m transform along axis 0 only; the 1/m of the
// unitary pair is folded into the mask.  The coil maps of coil c + 1 are
// loaded while coil c is transformed.
// MODE CA_APPLY  p = xin
//      CA_PCG    p = zs + beta p_old (beta from the rho partials), written to pn;
//                sigma = Re(p^H A p) partial
// PH AP_FUSED  everything in one launch
//    AP_PART   grid.z = ngroups workgroups per column tile; a slice with nc
//              coils uses gs = min(ngroups, ceil(nc / kpg)) of them (all
//              ngroups when kpg = 0), so that no workgroup of a batch with
//              uneven coil counts holds more than kpg coils; group z < gs
//              takes coils z, z + gs, ... and writes its partial data term to
//              dpart[z] (CA_PCG: group 0 also writes pn); groups z >= gs exit
//    AP_FIN    adds the slice's gs partial sums in group order, then the
//              diagonal terms and the mode's outputs (CA_PCG reads p back
//              from pn)
// ----------------------------------------------------------------------------
template <int M, int MODE, int PH, int TW = col_tile(M)>
__global__ __launch_bounds__((ApplyCfg<M, TW>::THREADS), (ApplyCfg<M, TW>::MIN_BLOCKS)) void k_col_apply(
    Ws w, int terms, int pk, double tol, const float2* __restrict__ xin, const float2* __restrict__ zsrc,
    const float2* __restrict__ pold, float2* __restrict__ pn, float2* __restrict__ out, int ngroups, int kpg,
    float2* __restrict__ dpart, long long dstride) {
  using Cfg = ApplyCfg<M, TW>;
  constexpr int NT = Cfg::NT, E = Cfg::E, T = Cfg::T, TH = Cfg::THREADS;
  constexpr int TS = T + 2;  // tile stride with the two halo columns
  constexpr int HP = (2 * M + TH - 1) / TH;
  constexpr bool DUAL = ApplyDual<M>::value;
  constexpr int LB = ColLay<T>::template size<M>;  // one exchange buffer
  __shared__ float2 lds[DUAL ? (2 * LB > M * TS ? 2 * LB : M * TS) : (LB > M * TS ? LB : M * TS)];
  __shared__ float2 s_tw[M];
  __shared__ double red[16];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  const int n = sd.n;
  const int gs = kpg > 0 ? min(ngroups, (sd.nc + kpg - 1) / kpg) : ngroups;  // this slice's coil groups
  if (PH == AP_PART && (int)blockIdx.z >= gs) return;
  const int j = threadIdx.x % T, t = threadIdx.x / T;
  const int j0 = xcd_tile(blockIdx.x, gridDim.x) * T;
  const int col = j0 + j;
  // CA_PCG in the finishing pass: p was written to pn by the partial pass
  const float2* __restrict__ xs = (MODE == CA_PCG ? (const float2*)pn : xin) + sd.img;

  int it = 0;
  float beta = 0.f;
  bool first = true;
  if (MODE == CA_PCG) {
    PcgState* st = w.st + s;
    if (st->done) return;
    int status;
    if (pcg_should_stop(w, s, sd.m, tol, &status)) {
      if (blockIdx.x == 0 && blockIdx.z == 0 && threadIdx.x == 0) pcg_mark_done(w, s, status, tol);
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
  stage_twiddles<M, TH>(s_tw, w.tw);

  // p for the tile (cyclic rows); the two halo columns are loaded with it,
  // or after the coil loop for narrow tiles (more halo values per thread)
  const float2* __restrict__ zs = zsrc + sd.img;
  const float2* __restrict__ po = pold + sd.img;
  const float* __restrict__ jc = w.jac + sd.img;
  float2 pv[E], ph[HP];
  auto load_halo = [&]() {
    const int jl = (j0 - 1 + n) % n, jr = (j0 + T) % n;
    int hoff[HP];
#pragma unroll
    for (int k = 0; k < HP; ++k) {
      const int h = threadIdx.x + k * TH;
      const int side = h / M, i = h % M;
      hoff[k] = h < 2 * M ? i * n + (side ? jr : jl) : 0;
    }
    if (MODE != CA_PCG || PH == AP_FIN) {
      if (PH != AP_PART) {
#pragma unroll
        for (int k = 0; k < HP; ++k) ph[k] = xs[hoff[k]];
      }
    } else if (PH == AP_FUSED) {
#pragma unroll
      for (int k = 0; k < HP; ++k) ph[k] = zs[hoff[k]];
      if (pk == PK_JACOBI) {
        float jh[HP];
#pragma unroll
        for (int k = 0; k < HP; ++k) jh[k] = jc[hoff[k]];
#pragma unroll
        for (int k = 0; k < HP; ++k) ph[k] = cscale(ph[k], jh[k]);
      }
      if (!first) {
        float2 oh[HP];
#pragma unroll
        for (int k = 0; k < HP; ++k) oh[k] = po[hoff[k]];
#pragma unroll
        for (int k = 0; k < HP; ++k) ph[k] = make_float2(ph[k].x + beta * oh[k].x, ph[k].y + beta * oh[k].y);
      }
    }
  };
  constexpr bool LATE_HALO = HP > 4 || M == 320;  // (320: registers, see the coil loop)
  if (MODE != CA_PCG || PH == AP_FIN) {
#pragma unroll
    for (int e = 0; e < E; ++e) pv[e] = xs[(t + NT * e) * n + col];
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) pv[e] = zs[(t + NT * e) * n + col];
    if (pk == PK_JACOBI) {
      float jv[E];
#pragma unroll
      for (int e = 0; e < E; ++e) jv[e] = jc[(t + NT * e) * n + col];
#pragma unroll
      for (int e = 0; e < E; ++e) pv[e] = cscale(pv[e], jv[e]);
    }
    if (!first) {
      float2 ov[E];
#pragma unroll
      for (int e = 0; e < E; ++e) ov[e] = po[(t + NT * e) * n + col];
#pragma unroll
      for (int e = 0; e < E; ++e) pv[e] = make_float2(pv[e].x + beta * ov[e].x, pv[e].y + beta * ov[e].y);
    }
    if (PH == AP_FUSED || blockIdx.z == 0) {
      float2* __restrict__ pno = pn + sd.img;
#pragma unroll
      for (int e = 0; e < E; ++e) pno[(t + NT * e) * n + col] = pv[e];
    }
  }
  if (!LATE_HALO) load_halo();
  // data term sum_c conj(S_c) F^H R F (S_c p), coil maps of c + 1 in flight.
  // AP_PART: coils c = z, z + gs, ... of group z = blockIdx.z, result to
  // dpart[z]; AP_FIN: the groups' partial sums added in group order.
  float2 acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = make_float2(0.f, 0.f);
  const int c0 = PH == AP_PART ? (int)blockIdx.z : 0;
  const int cstep = PH == AP_PART ? gs : 1;
  if (PH == AP_FIN) {
    for (int gidx = 0; gidx < gs; ++gidx) {
      const float2* __restrict__ dp = dpart + gidx * dstride + sd.img;
#pragma unroll
      for (int e = 0; e < E; ++e) acc[e] = cadd(acc[e], dp[(t + NT * e) * n + col]);
    }
  } else if ((terms & TERM_DATA) && c0 < sd.nc) {
    const uint8_t* mk = w.mask + sd.mask;
    unsigned mbits = 0u;  // bit e: frequency row t + NT e sampled
#pragma unroll
    for (int e = 0; e < E; ++e) mbits |= (mk[t + NT * e] ? 1u : 0u) << e;
    const float inv_m = 1.0f / M;
    float msc[E];  // mask / m per frequency row t + NT e
#pragma unroll
    for (int e = 0; e < E; ++e) msc[e] = ((mbits >> e) & 1u) ? inv_m : 0.f;
    const int plane = M * n;
    // coil c's maps for this thread's rows, by buffer loads: the resource
    // (the coil's plane) and the per-element offsets are wave-uniform, so the
    // addresses cost no vector instructions
    const int voff = (t * n + col) * (int)sizeof(float2);
    auto load_maps = [&](float2(&dst)[E], int c) {
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(w.sens + sd.coil + (long long)c * plane), (short)0, plane * (int)sizeof(float2), 0x00020000);
#pragma unroll
      for (int e = 0; e < E; ++e)
        dst[e] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, NT * e * n * 8, 0));
    };
    // the next coil's maps are prefetched, except at length 1024, where the
    // extra registers would spill, and at 320, where the registers they free
    // (with the halo loaded late) give two waves per SIMD instead of one
    constexpr bool PREFETCH = M < 1024 && M != 320;
    // one coil: S_c p -> FFT -> mask / m -> IFFT -> += conj(S_c) (.); `cur`
    // holds S_c, and with PF `nxt` receives the maps of coil pf once S_c p is
    // formed, so that the load runs during the transforms.  PF is a template
    // argument: a conditional load would make the compiler wait for every
    // load in flight before the first use of `cur`.
    auto coil_step = [&](auto pf_tag, const float2(&cur)[E], float2(&nxt)[E], int pf) {
      constexpr bool PF = decltype(pf_tag)::value;
      float2 v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = cmul(cur[e], pv[e]);
      if constexpr (PF) load_maps(nxt, pf);
      // the mask (with the 1/m of the unitary pair) scales the inverse
      // transform's inputs inside its first stage
      if constexpr (DUAL) {
        // exchanges alternate between the two buffers across both transforms
        constexpr bool odd = (kExchanges<M> & 1) != 0;
        fft_dual<M, -1, ColLay<T>>(v, t, lds, lds + LB, j, s_tw);
        fft_in_scaled<M, +1, ColLay<T>, true>(v, msc, t, odd ? lds + LB : lds, odd ? lds : lds + LB, j, s_tw);
      } else {
        fft<M, -1, ColLay<T>>(v, t, lds, j, s_tw);
        fft_in_scaled<M, +1, ColLay<T>, false>(v, msc, t, lds, lds, j, s_tw);
      }
#pragma unroll
      for (int e = 0; e < E; ++e) acc[e] = cadd(acc[e], cconjmul(cur[e], v[e]));
    };
    const std::integral_constant<bool, true> with_prefetch;
    const std::integral_constant<bool, false> without;
    float2 sa[E], sb[E];
    load_maps(sa, c0);
    // lengths up to 256 with 16 or fewer elements per thread: two coils per
    // trip; the longer register files of 224 keep one coil per trip (four
    // inlined transforms would spill)
    constexpr bool PAIRS = PREFETCH && E <= 16;
    if constexpr (PAIRS) {
      // coils k = 0 .. K-1 of this workgroup (c0 + k cstep); two per trip,
      // the map buffers swapping roles (no copies); the last one or two
      // outside the loop, where nothing is left to prefetch
      const int K = (sd.nc - c0 + cstep - 1) / cstep;
      int k = 0;
      for (; k + 2 < K; k += 2) {
        coil_step(with_prefetch, sa, sb, c0 + (k + 1) * cstep);
        coil_step(with_prefetch, sb, sa, c0 + (k + 2) * cstep);
      }
      if (k + 2 == K) {
        coil_step(with_prefetch, sa, sb, c0 + (k + 1) * cstep);
        coil_step(without, sb, sa, 0);
      } else {
        coil_step(without, sa, sb, 0);
      }
    } else {
      for (int c = c0; c < sd.nc; c += cstep) {
        if (!PREFETCH && c != c0) load_maps(sa, c);
        // unconditional (the last trip reloads its own maps): a conditional
        // load makes the compiler wait on it before the transforms
        if (PREFETCH) load_maps(sb, c + cstep < sd.nc ? c + cstep : c);
        coil_step(without, sa, sb, 0);
        if (PREFETCH) {
#pragma unroll
          for (int e = 0; e < E; ++e) sa[e] = sb[e];
        }
      }
    }
  }
  if (PH == AP_PART) {
    float2* __restrict__ dp = dpart + (long long)blockIdx.z * dstride + sd.img;
#pragma unroll
    for (int e = 0; e < E; ++e) dp[(t + NT * e) * n + col] = acc[e];
    return;
  }
  if (LATE_HALO) load_halo();
  __syncthreads();  // the FFTs are done with the LDS buffer

  // Fourier-diagonal terms lam (D_x^H D_x + D_y^H D_y) p + gam p on the tile
#pragma unroll
  for (int e = 0; e < E; ++e) lds[(t + NT * e) * TS + j + 1] = pv[e];
#pragma unroll
  for (int k = 0; k < HP; ++k) {
    const int h = threadIdx.x + k * TH;
    if (h < 2 * M) lds[(h % M) * TS + (h / M ? T + 1 : 0)] = ph[k];
  }
  __syncthreads();
  const float mu = sd.mu, lam = sd.lam, gam = sd.gam;
  float2 q[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = t + NT * e;
    float2 a = make_float2(mu * acc[e].x, mu * acc[e].y);
    if (terms & TERM_TV) {
      const int iu = (i - 1 + M) % M, id = (i + 1) % M;
      const float2 c = lds[i * TS + j + 1];
      const float2 u = lds[iu * TS + j + 1], d = lds[id * TS + j + 1];
      const float2 l = lds[i * TS + j], r = lds[i * TS + j + 2];
      a = make_float2(a.x + lam * (4.f * c.x - u.x - d.x - l.x - r.x), a.y + lam * (4.f * c.y - u.y - d.y - l.y - r.y));
    }
    if (terms & TERM_GAMMA) a = make_float2(a.x + gam * pv[e].x, a.y + gam * pv[e].y);
    q[e] = a;
  }

  float2* __restrict__ o = out + sd.img;
  double sig = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    o[(t + NT * e) * n + col] = q[e];
    sig += (double)pv[e].x * (double)q[e].x + (double)pv[e].y * (double)q[e].y;
  }
  if (MODE == CA_PCG) {
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
//   RU_UPDATE: alpha = rho / sigma; x += alpha pn; r -= alpha q
// Circulant / learned: t = row-FFT(r).  None / Jacobi: rho' = Re(r^H z)
// partial with z = r or z = r / diag(A).
// ----------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void k_row_update(Ws w, int mode, int pk,
                                                                   const float2* __restrict__ b,
                                                                   const float2* __restrict__ q, float2* x, float2* r,
                                                                   const float2* __restrict__ pn, float2* p,
                                                                   float2* __restrict__ tout, int maxit,
                                                                   const int* __restrict__ maxit_ps) {
  constexpr int NT = RowCfg<N>::NT, E = RowCfg<N>::E;
  __shared__ float2 lds[RowCfg<N>::LDS];
  __shared__ float2 s_tw[N];
  __shared__ double red[16];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  PcgState* st = w.st + s;
  const int t = threadIdx.x % NT, rr_ = threadIdx.x / NT;
  const int i = blockIdx.x * kRowRR + rr_;
  const long long rowbase = sd.img + (long long)i * N;
  if (pk != PK_NONE && pk != PK_JACOBI) stage_twiddles<N, RowCfg<N>::THREADS>(s_tw, w.tw);

  int it = 0;
  float alpha = 0.f;
  if (mode == RU_SETUP && blockIdx.x == 0 && threadIdx.x == 0) {
    // a new solve: reset the slice's PCG state (nothing reads it before the
    // set-up's stop test, which follows this kernel)
    PcgState ns;
    ns.it_a = 0;
    ns.it_r = 0;
    ns.done = 0;
    ns.status = 0;
    ns.iters = 0;
    ns.maxit = maxit_ps ? maxit_ps[s] : maxit;
    ns.relres = 0.0;
    *st = ns;
  }
  if (mode == RU_UPDATE) {
    if (st->done) return;
    it = st->it_r;
    // sigma partials: one per column tile (line masks) or row tile (2D masks)
    const int nrt = sd.m / kRowRR, nct = sd.mask_kind == 0 ? sd.ctiles : nrt;
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

  // every load of the row is issued before the first store (x and r are
  // written in place), so the loads of all elements are in flight together
  float2 v[E];
  double rrp = 0.0, bbp = 0.0, rhop = 0.0;
  if (mode == RU_UPDATE) {
    float2 pv[E], xv[E], qv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const long long idx = rowbase + t + NT * e;
      pv[e] = pn[idx];
      xv[e] = x[idx];
      v[e] = r[idx];
      qv[e] = q[idx];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const long long idx = rowbase + t + NT * e;
      x[idx] = make_float2(xv[e].x + alpha * pv[e].x, xv[e].y + alpha * pv[e].y);
      v[e] = make_float2(v[e].x - alpha * qv[e].x, v[e].y - alpha * qv[e].y);
      r[idx] = v[e];
    }
  } else {
    float2 bv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const long long idx = rowbase + t + NT * e;
      bv[e] = b[idx];
      v[e] = q[idx];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      v[e] = csub(bv[e], v[e]);
      bbp += (double)bv[e].x * bv[e].x + (double)bv[e].y * bv[e].y;
      r[rowbase + t + NT * e] = v[e];
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const double a2 = (double)v[e].x * v[e].x + (double)v[e].y * v[e].y;
    rrp += a2;
    if (pk == PK_JACOBI) rhop += (double)w.jac[rowbase + t + NT * e] * a2;
    if (pk == PK_NONE) rhop += a2;
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
    fft<N, -1, RowLay<N>>(v, t, lds, rr_, s_tw);
#pragma unroll
    for (int e = 0; e < E; ++e) tout[rowbase + t + NT * e] = v[e];
  }
  if (mode == RU_UPDATE && blockIdx.x == 0 && threadIdx.x == 0) st->it_a = it + 1;
}

// ----------------------------------------------------------------------------
// Middle pass of M^{-1} = F^H diag(1/k) F: column FFT, scale by 1/(k m n),
// inverse column FFT, in place.  With `check` the stop rule is tested first:
// check 1 inside the iteration, check 2 at the set-up, where a zero
// right-hand side also stops the solve with x = 0 (every workgroup clears
// its own columns of x; the control block, just reset by the set-up, is not
// read, so all workgroups take the same decision).  use_state = 0 ignores the
// PCG control block (stand-alone M^{-1}).
// ----------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(ColCfg<M>::THREADS) void k_col_precond(Ws w, int use_state, int check, double tol,
                                                                     float2* __restrict__ tbuf,
                                                                     float2* __restrict__ x) {
  constexpr int NT = ColCfg<M>::NT, E = ColCfg<M>::E, T = ColCfg<M>::T;
  __shared__ float2 lds[ColLay<T>::template size<M>];
  __shared__ float2 s_tw[M];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  const int n = sd.n;
  const int j = threadIdx.x % T, t = threadIdx.x / T;
  const int col = xcd_tile(blockIdx.x, gridDim.x) * T + j;
  const long long base = sd.img;
  if (use_state) {
    if (check != 2 && w.st[s].done) return;
    int status;
    bool zero_x = false;
    if (check == 2) {
      const double bb = part_sum(part_ptr(w.part, s, P_BB), sd.m / kRowRR);
      zero_x = bb == 0.0;
    }
    if (zero_x || (check && pcg_should_stop(w, s, sd.m, tol, &status))) {
      if (zero_x) {
        status = 1;
#pragma unroll
        for (int e = 0; e < E; ++e) x[base + (long long)(t + NT * e) * n + col] = make_float2(0.f, 0.f);
      }
      if (blockIdx.x == 0 && threadIdx.x == 0) pcg_mark_done(w, s, status, tol);
      return;
    }
  }
  stage_twiddles<M, ColCfg<M>::THREADS>(s_tw, w.tw);
  float2 v[E];
  float kv[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = tbuf[base + (long long)(t + NT * e) * n + col];
#pragma unroll
  for (int e = 0; e < E; ++e) kv[e] = w.kinv[base + (long long)(t + NT * e) * n + col];
  fft<M, -1, ColLay<T>>(v, t, lds, j, s_tw);
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = cscale(v[e], kv[e]);
  fft<M, +1, ColLay<T>>(v, t, lds, j, s_tw);
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
  __shared__ float2 s_tw[N];
  __shared__ double red[16];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  PcgState* st = w.st + s;
  if (st->done) return;
  const int t = threadIdx.x % NT, rr_ = threadIdx.x / NT;
  const int i = blockIdx.x * kRowRR + rr_;
  const long long rowbase = sd.img + (long long)i * N;
  stage_twiddles<N, RowCfg<N>::THREADS>(s_tw, w.tw);
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = tbuf[rowbase + t + NT * e];
  fft<N, +1, RowLay<N>>(v, t, lds, rr_, s_tw);
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
// Plain row FFT (unnormalised).  ncoil_mode 1: loop over the slice's coils on
// coil-shaped buffers, zeroing unsampled k-space first (R y before F^H; the
// unsampled lines of a line mask are skipped, left unwritten in `out`);
// ncoil_mode 2: the same loop without the mask.
// ----------------------------------------------------------------------------
template <int N, int DIR>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void k_row_fft(Ws w, int ncoil_mode, const float2* __restrict__ in,
                                                                float2* __restrict__ out) {
  constexpr int NT = RowCfg<N>::NT, E = RowCfg<N>::E;
  __shared__ float2 lds[RowCfg<N>::LDS];
  __shared__ float2 s_tw[N];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  const int t = threadIdx.x % NT, rr_ = threadIdx.x / NT;
  const int i = blockIdx.x * kRowRR + rr_;
  stage_twiddles<N, RowCfg<N>::THREADS>(s_tw, w.tw);
  const int ncoil = ncoil_mode ? sd.nc : 1;
  const long long plane = (long long)sd.m * N;
  const uint8_t* mk = w.mask + sd.mask;
  // an unsampled line of a line mask is neither read nor written: the
  // column pass that follows treats it as zero
  // (the next coil's row is loaded while this one is transformed, except at
  // length 1024, where 1024-thread workgroups leave no registers for it)
  constexpr bool PF = N < 1024;
  const bool dead_row = ncoil_mode == 1 && sd.mask_kind == 0 && mk[i] == 0;
  const long long row0 = (ncoil_mode ? sd.coil : sd.img) + (long long)i * N;
  auto load_row = [&](long long rowbase, float2 (&v)[E]) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      float2 a = make_float2(0.f, 0.f);
      if (!dead_row) a = in[rowbase + t + NT * e];
      if (ncoil_mode == 1 && sd.mask_kind != 0 && mk[(long long)i * N + t + NT * e] == 0) a = make_float2(0.f, 0.f);
      v[e] = a;
    }
  };
  float2 v[E], vn[E];
  load_row(row0, v);
  for (int c = 0; c < ncoil; ++c) {
    const long long rowbase = row0 + c * plane;
    if (!PF && c > 0) load_row(rowbase, v);
    // (unconditional: the last trip reloads its own row, which keeps the
    // compiler from waiting on the loads before the transform)
    if (PF) load_row(rowbase + (c + 1 < ncoil ? plane : 0), vn);
    fft<N, DIR, RowLay<N>>(v, t, lds, rr_, s_tw);
    if (!dead_row) {
#pragma unroll
      for (int e = 0; e < E; ++e) out[rowbase + t + NT * e] = v[e];
    }
    if (PF) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = vn[e];
    }
  }
}

// Plain column FFT (unnormalised), image-shaped buffers.
template <int M, int DIR>
__global__ __launch_bounds__(ColCfg<M>::THREADS) void k_col_fft(Ws w, const float2* __restrict__ in,
                                                                float2* __restrict__ out) {
  constexpr int NT = ColCfg<M>::NT, E = ColCfg<M>::E, T = ColCfg<M>::T;
  __shared__ float2 lds[ColLay<T>::template size<M>];
  __shared__ float2 s_tw[M];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  const int n = sd.n;
  const int j = threadIdx.x % T, t = threadIdx.x / T;
  const int col = blockIdx.x * T + j;
  stage_twiddles<M, ColCfg<M>::THREADS>(s_tw, w.tw);
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = in[sd.img + (long long)(t + NT * e) * n + col];
  fft<M, DIR, ColLay<T>>(v, t, lds, j, s_tw);
#pragma unroll
  for (int e = 0; e < E; ++e) out[sd.img + (long long)(t + NT * e) * n + col] = v[e];
}

// ----------------------------------------------------------------------------
// Split Bregman initialisation (Algorithm 1, step 1 and the data part of the
// first right-hand side): per coil, finish the 2D inverse FFT of R y_c along
// axis 0 (the row pass already ran), scale to the unitary F^H, and form
//   g1 = mu sum_c conj(S_c) m_c,   x = sqrt(sum_c |m_c|^2)   (root sum of squares)
// g = g1, and the first right-hand side, g1 as well (d - b = 0 at the start).
// ----------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(ColCfg<M>::THREADS) void k_col_sb_init(Ws w, const float2* __restrict__ coil_rows,
                                                                     float2* __restrict__ g1, float2* __restrict__ g,
                                                                     float2* __restrict__ rhs,
                                                                     float2* __restrict__ x) {
  constexpr int NT = ColCfg<M>::NT, E = ColCfg<M>::E, T = ColCfg<M>::T;
  __shared__ float2 lds[ColLay<T>::template size<M>];
  __shared__ float2 s_tw[M];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  const int n = sd.n;
  const int j = threadIdx.x % T, t = threadIdx.x / T;
  const int col = blockIdx.x * T + j;
  stage_twiddles<M, ColCfg<M>::THREADS>(s_tw, w.tw);
  const float scale = 1.0f / sqrtf((float)M * (float)n);
  float2 acc[E];
  float sos[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    acc[e] = make_float2(0.f, 0.f);
    sos[e] = 0.f;
  }
  // line masks: the row pass left unsampled lines unwritten (they are zero)
  unsigned live = ~0u;
  if (sd.mask_kind == 0) {
    const uint8_t* mk = w.mask + sd.mask;
    live = 0u;
#pragma unroll
    for (int e = 0; e < E; ++e) live |= (mk[t + NT * e] ? 1u : 0u) << e;
  }
  // the coil's maps are requested before its transform, the next coil's
  // k-space rows while it runs
  const long long plane = (long long)M * n, off = (long long)t * n + col;
  float2 v[E], vn[E];
#pragma unroll
  for (int e = 0; e < E; ++e)
    v[e] = ((live >> e) & 1u) ? coil_rows[sd.coil + off + (long long)NT * e * n] : make_float2(0.f, 0.f);
  for (int c = 0; c < sd.nc; ++c) {
    const long long cb = sd.coil + c * plane;
    float2 sv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) sv[e] = w.sens[cb + off + (long long)NT * e * n];
    {
      // unconditional (the last trip reloads its own rows), see k_row_fft
      const long long nx = c + 1 < sd.nc ? plane : 0;
#pragma unroll
      for (int e = 0; e < E; ++e)
        vn[e] = ((live >> e) & 1u) ? coil_rows[cb + nx + off + (long long)NT * e * n] : make_float2(0.f, 0.f);
    }
    fft<M, +1, ColLay<T>>(v, t, lds, j, s_tw);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const float2 mc = cscale(v[e], scale);
      acc[e] = cadd(acc[e], cconjmul(sv[e], mc));
      sos[e] += cabs2(mc);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = vn[e];
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const long long idx = sd.img + (long long)(t + NT * e) * n + col;
    const float2 gv = cscale(acc[e], sd.mu);
    g1[idx] = gv;
    g[idx] = gv;
    rhs[idx] = gv;
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
  // the next coil's maps are loaded while this coil is transformed
  const float2* __restrict__ S = w.sens + sd.coil + (long long)t * n + col;
  const long long plane = (long long)M * n;
  float2 sv[E], sn[E];
#pragma unroll
  for (int e = 0; e < E; ++e) sv[e] = S[(long long)NT * e * n];
  for (int c = 0; c < sd.nc; ++c) {
    {
      // unconditional (the last trip reloads its own maps), see k_row_fft
      const int cn = c + 1 < sd.nc ? c + 1 : c;
#pragma unroll
      for (int e = 0; e < E; ++e) sn[e] = S[cn * plane + (long long)NT * e * n];
    }
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      v[e] = sv[e];
      en[e] += cabs2(v[e]);
    }
    fft<M, -1, ColLay<T>>(v, t, lds, j, s_tw);
#pragma unroll
    for (int e = 0; e < E; ++e) pw[e] += (double)v[e].x * v[e].x + (double)v[e].y * v[e].y;
#pragma unroll
    for (int e = 0; e < E; ++e) sv[e] = sn[e];
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

// ----------------------------------------------------------------------------
// Unitary k-space coil energy sum_c |F s_c|^2 per pixel: the column pass of the
// 2D transform of every coil map (the row pass already ran), squared
// magnitudes summed over coils, scaled by 1 / N.
// ----------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(ColCfg<M>::THREADS) void k_col_coil_energy(Ws w, const float2* __restrict__ coil_rows,
                                                                        float* __restrict__ energy) {
  constexpr int NT = ColCfg<M>::NT, E = ColCfg<M>::E, T = ColCfg<M>::T;
  __shared__ float2 lds[ColLay<T>::template size<M>];
  __shared__ float2 s_tw[M];
  const int s = w.group[blockIdx.y];
  const SliceDev sd = w.sl[s];
  const int n = sd.n;
  const int j = threadIdx.x % T, t = threadIdx.x / T;
  const int col = blockIdx.x * T + j;
  stage_twiddles<M, ColCfg<M>::THREADS>(s_tw, w.tw);
  float en[E];
#pragma unroll
  for (int e = 0; e < E; ++e) en[e] = 0.f;
  for (int c = 0; c < sd.nc; ++c) {
    const long long cb = sd.coil + (long long)c * M * n;
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = coil_rows[cb + (long long)(t + NT * e) * n + col];
    fft<M, -1, ColLay<T>>(v, t, lds, j, s_tw);
#pragma unroll
    for (int e = 0; e < E; ++e) en[e] += cabs2(v[e]);
  }
  const float inv = 1.0f / ((float)M * (float)n);
#pragma unroll
  for (int e = 0; e < E; ++e) energy[sd.img + (long long)(t + NT * e) * n + col] = en[e] * inv;
}

// ============================================================== launchers

template <int M, int PH, int TW = col_tile(M)>
void launch_col_apply_phase(dim3 grid, const Launch& L, const Ws& w, int mode, int terms, int pk, double tol,
                            const float2* xin, const float2* zsrc, const float2* pold, float2* pn, float2* out,
                            int ngroups, int kpg, float2* dpart, long long dstride) {
  const dim3 block(ApplyCfg<M, TW>::THREADS);
  if (mode == CA_PCG)
    hipLaunchKernelGGL((k_col_apply<M, CA_PCG, PH, TW>), grid, block, 0, L.stream, w, terms, pk, tol, xin, zsrc,
                       pold, pn, out, ngroups, kpg, dpart, dstride);
  else
    hipLaunchKernelGGL((k_col_apply<M, CA_APPLY, PH, TW>), grid, block, 0, L.stream, w, terms, pk, tol, xin, zsrc,
                       pold, pn, out, ngroups, kpg, dpart, dstride);
}

bool apply_tile_ok(int m, int n, int tile) {
  if (tile == col_tile(m)) return true;
  if (tile != apply_tile_alt(m, 0) && tile != apply_tile_alt(m, 1)) return false;
  return n % tile == 0 && n / tile <= kPartMax;
}

hipError_t launch_col_apply(const Launch& L, const Ws& w, int mode, int terms, int pk, double tol,
                            const float2* xin, const float2* zsrc, const float2* pold, float2* pn, float2* out,
                            int ngroups, float2* dpart, long long dstride, int tile, int ncmax) {
  const int split = (ngroups > 1 && (terms & TERM_DATA)) ? ngroups : 1;
  // coils per partial workgroup: the largest slice's split (0: every slice split ngroups ways)
  const int kpg = split > 1 && ncmax > 0 ? (ncmax + split - 1) / split : 0;
  if (split > 1 && !dpart) return hipErrorInvalidValue;
  if (tile == 0) tile = col_tile(L.m);
  // a coil split runs with the default tiles only
  if (!apply_tile_ok(L.m, L.n, tile) || (split > 1 && tile != col_tile(L.m))) return hipErrorInvalidValue;
  const dim3 grid(L.n / tile, L.count);
  switch (L.m) {
#define PICS_CASE(M)                                                                                            \
  case M:                                                                                                       \
    if (tile == apply_tile_alt(M, 0)) {                                                                         \
      launch_col_apply_phase<M, AP_FUSED, apply_tile_alt(M, 0)>(grid, L, w, mode, terms, pk, tol, xin, zsrc,     \
                                                               pold, pn, out, 1, 0, dpart, dstride);           \
    } else if (tile == apply_tile_alt(M, 1)) {                                                                  \
      launch_col_apply_phase<M, AP_FUSED, apply_tile_alt(M, 1)>(grid, L, w, mode, terms, pk, tol, xin, zsrc,     \
                                                               pold, pn, out, 1, 0, dpart, dstride);           \
    } else if (split == 1) {                                                                                    \
      launch_col_apply_phase<M, AP_FUSED>(grid, L, w, mode, terms, pk, tol, xin, zsrc, pold, pn, out, 1, 0,      \
                                          dpart, dstride);                                                     \
    } else {                                                                                                    \
      launch_col_apply_phase<M, AP_PART>(dim3(grid.x, grid.y, split), L, w, mode, terms, pk, tol, xin, zsrc,    \
                                         pold, pn, out, split, kpg, dpart, dstride);                           \
      const hipError_t e = hipGetLastError();                                                                   \
      if (e != hipSuccess) return e;                                                                            \
      launch_col_apply_phase<M, AP_FIN>(grid, L, w, mode, terms, pk, tol, xin, zsrc, pold, pn, out, split, kpg, \
                                        dpart, dstride);                                                       \
    }                                                                                                           \
    break;
    PICS_FFT_SIZES(PICS_CASE)
#undef PICS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_row_update(const Launch& L, const Ws& w, int mode, int pk, const float2* b, const float2* q,
                             float2* x, float2* r, const float2* pn, float2* p, float2* t, int maxit,
                             const int* maxit_ps) {
  const dim3 grid(L.m / kRowRR, L.count);
  switch (L.n) {
#define PICS_CASE(N)                                                                                      \
  case N:                                                                                                 \
    hipLaunchKernelGGL(k_row_update<N>, grid, dim3(RowCfg<N>::THREADS), 0, L.stream, w, mode, pk, b, q, x, \
                       r, pn, p, t, maxit, maxit_ps);                                                     \
    break;
    PICS_FFT_SIZES(PICS_CASE)
#undef PICS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_col_precond(const Launch& L, const Ws& w, int use_state, int check, double tol, float2* t,
                              float2* x) {
  const dim3 grid(L.n / col_tile(L.m), L.count);
  switch (L.m) {
#define PICS_CASE(M)                                                                                           \
  case M:                                                                                                      \
    hipLaunchKernelGGL(k_col_precond<M>, grid, dim3(ColCfg<M>::THREADS), 0, L.stream, w, use_state, check, tol, \
                       t, x);                                                                                  \
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
  const dim3 grid(L.n / col_tile(L.m), L.count);
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
                              float2* rhs, float2* x) {
  const dim3 grid(L.n / col_tile(L.m), L.count);
  switch (L.m) {
#define PICS_CASE(M)                                                                                                  \
  case M:                                                                                                             \
    hipLaunchKernelGGL(k_col_sb_init<M>, grid, dim3(ColCfg<M>::THREADS), 0, L.stream, w, coil_rows, g1, g, rhs, x); \
    break;
    PICS_FFT_SIZES(PICS_CASE)
#undef PICS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_col_coil_power(const Launch& L, const Ws& w, double* pbar, float* energy) {
  const dim3 grid(L.n / col_tile(L.m), L.count);
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

hipError_t launch_col_coil_energy(const Launch& L, const Ws& w, const float2* coil_rows, float* energy) {
  const dim3 grid(L.n / col_tile(L.m), L.count);
  switch (L.m) {
#define PICS_CASE(M)                                                                                               \
  case M:                                                                                                          \
    hipLaunchKernelGGL(k_col_coil_energy<M>, grid, dim3(ColCfg<M>::THREADS), 0, L.stream, w, coil_rows, energy); \
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

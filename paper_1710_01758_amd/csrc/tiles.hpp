// Tile configurations and device helpers shared by the FFT-pass kernels.
//
// Column tiles: a workgroup owns T = 16 adjacent columns of one slice and all
// m rows; thread (t, j) holds rows t + NT e of column j (cyclic layout), so a
// length-m transform along axis 0 runs in registers + LDS.  Row tiles: a
// workgroup owns 16 rows, thread (t, r) holds columns t + NT e of row r.
#pragma once

#include "fft.hpp"
#include "internal.hpp"

namespace pics {

template <int M, class P = Plan<M>>
struct ColCfg {
  static constexpr int NT = P::NT;
  static constexpr int E = M / NT;
  static constexpr int T = col_tile(M);
  static constexpr int THREADS = NT * T;
};

// The fused operator's column tiles; lengths up to 256 give each transform
// exchange its own LDS buffer (two buffers used in turn, so a barrier after
// reading an exchange is not needed).
// TW: columns per tile (the default col_tile(M), or one of the autotuner's
// alternatives, apply_tile_alt).
template <int M, int TW = col_tile(M)>
struct ApplyCfg {
  static constexpr int NT = Plan<M>::NT;
  static constexpr int E = M / NT;
  static constexpr int T = TW;
  static constexpr int THREADS = NT * T;
  // workgroups per CU the register allocation must allow: two waves per
  // SIMD at 320 and 512 with the default tiles; the alternative widths ask
  // for two waves per SIMD as well (at most 256 registers per lane)
  static constexpr int MIN_BLOCKS = TW == col_tile(M) ? (M == 320 || M == 512 ? 2 : 1)
                                                      : (512 / THREADS > 0 ? 512 / THREADS : 1);
};
template <int M>
struct ApplyDual { static constexpr bool value = M <= 256; };
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

// Copy this length's twiddle table into LDS so that the FFT stages read it
// with LDS instructions (the global-load counter then only tracks data).
template <int N, int TH>
__device__ __forceinline__ void stage_twiddles(float2* s_tw, const float2* __restrict__ tw_global) {
  const float2* __restrict__ src = tw_global + tw_offset(N);
  for (int k = threadIdx.x; k < N; k += TH) s_tw[k] = src[k];
}

}  // namespace pics

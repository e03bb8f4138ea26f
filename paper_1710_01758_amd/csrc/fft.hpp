// Mixed-radix complex FFTs staged through LDS (gfx950).
//
// A length-N transform is carried by NT threads; thread t holds E = N / NT
// elements in registers in the "cyclic" layout v[e] = element t + NT * e.
// A plan is a list of radices R_1 .. R_s with product N, each dividing E.
// Stage s (span Ns = R_1 ... R_{s-1}) is a self-sorting Stockham pass: the
// thread computes E / R_s butterflies b = t + NT q, reading the cyclic inputs
// v[q + r E/R_s], scaling input r by w_{Ns R}^{(b mod Ns) r}, applying an
// in-register radix-R DFT and writing output r to position
// (b / Ns) Ns R + (b mod Ns) + r Ns.  Between stages the outputs go through
// LDS and come back in the cyclic layout; the last stage's outputs land
// directly in the cyclic layout in registers, in natural frequency order.
// No normalisation is applied (forward = exp(-2 pi i / N) kernel, inverse =
// exp(+2 pi i / N)).
#pragma once

#include "common.hpp"

namespace pics {

// ----------------------------------------------------- twiddle multiplies

// a * exp(DIR 2 pi i K / R), with the exact special cases of multiples of
// 45 degrees.
template <int R, int K, int DIR>
__device__ __forceinline__ float2 tw_mul(float2 a) {
  constexpr int k = ((K % R) + R) % R;
  if constexpr (k == 0) {
    return a;
  } else if constexpr ((8 * k) % R == 0) {
    constexpr int oct = (8 * k) / R;  // multiple of 45 degrees, 1..7
    constexpr float h = 0.70710678118654752440f;
    if constexpr (oct == 4) {
      return make_float2(-a.x, -a.y);
    } else if constexpr (oct == 2) {
      return cmul_i(a, float(DIR));
    } else if constexpr (oct == 6) {
      return cmul_i(a, -float(DIR));
    } else {
      // (c + i DIR s) with |c| = |s| = h
      constexpr float c = (oct == 1 || oct == 7) ? h : -h;
      constexpr float s = (oct == 1 || oct == 3) ? h : -h;
      constexpr float sd = s * float(DIR);
      return make_float2(c * a.x - sd * a.y, c * a.y + sd * a.x);
    }
  } else {
    constexpr float c = TwC<R, k, DIR>::re;
    constexpr float s = TwC<R, k, DIR>::im;
    return make_float2(c * a.x - s * a.y, c * a.y + s * a.x);
  }
}

// ------------------------------------------------- in-register small DFTs

template <int R>
struct Split;  // R = P * Q for the composite sizes
template <> struct Split<8> { static constexpr int P = 4, Q = 2; };
template <> struct Split<12> { static constexpr int P = 4, Q = 3; };
template <> struct Split<16> { static constexpr int P = 4, Q = 4; };
template <> struct Split<20> { static constexpr int P = 4, Q = 5; };
template <> struct Split<24> { static constexpr int P = 8, Q = 3; };
template <> struct Split<28> { static constexpr int P = 4, Q = 7; };
template <> struct Split<32> { static constexpr int P = 8, Q = 4; };
template <> struct Split<40> { static constexpr int P = 8, Q = 5; };
template <> struct Split<64> { static constexpr int P = 8, Q = 8; };

// Odd multiples of 45 degrees: exp(DIR 2 pi i K / R) = h (c + i DIR s) with
// c, s = +-1 and h = 1/sqrt(2).  tw45_unscaled returns a (c + i DIR s)
// (adds only); the caller owes the factor h, which the second-level DFT
// below folds into fused multiply-adds.
template <int R, int K>
struct Tw45 {
  static constexpr int k = ((K % R) + R) % R;
  static constexpr bool value = k != 0 && (8 * k) % R == 0 && (((8 * k) / R) & 1) == 1;
};
template <int R, int K, int DIR>
__device__ __forceinline__ float2 tw45_unscaled(float2 a) {
  constexpr int oct = (8 * Tw45<R, K>::k) / R;  // 1, 3, 5 or 7
  constexpr float c = (oct == 1 || oct == 7) ? 1.f : -1.f;
  constexpr float sd = ((oct == 1 || oct == 3) ? 1.f : -1.f) * float(DIR);
  return make_float2(c * a.x - sd * a.y, c * a.y + sd * a.x);
}

constexpr float kH = 0.70710678118654752440f;

__device__ __forceinline__ float2 cfma(float s, float2 a, float2 b) {  // s a + b
  return make_float2(__builtin_fmaf(s, a.x, b.x), __builtin_fmaf(s, a.y, b.y));
}

template <int R, int DIR>
struct Dft;

// DFT of Q points whose inputs flagged in SM (bit n) still owe a factor h.
// The two patterns the radix-4 and radix-2 second levels meet (c2 alone; c1
// and c3 together) fold h into fused multiply-adds; any other pattern
// multiplies first.
template <int Q, int DIR, int SM>
struct DftScaled {
  static __device__ __forceinline__ void run(float2 (&c)[Q]) {
#pragma unroll
    for (int n = 0; n < Q; ++n)
      if ((SM >> n) & 1) c[n] = cscale(c[n], kH);
    Dft<Q, DIR>::run(c);
  }
};
template <int DIR>
struct DftScaled<2, DIR, 2> {
  static __device__ __forceinline__ void run(float2 (&c)[2]) {
    const float2 t = c[0];
    c[0] = cfma(kH, c[1], t);
    c[1] = cfma(-kH, c[1], t);
  }
};
template <int DIR>
struct DftScaled<4, DIR, 4> {  // c2 owes h
  static __device__ __forceinline__ void run(float2 (&a)[4]) {
    const float2 s02 = cfma(kH, a[2], a[0]), d02 = cfma(-kH, a[2], a[0]);
    const float2 s13 = cadd(a[1], a[3]), d13 = csub(a[1], a[3]);
    const float2 j13 = cmul_i(d13, float(DIR));
    a[0] = cadd(s02, s13);
    a[2] = csub(s02, s13);
    a[1] = cadd(d02, j13);
    a[3] = csub(d02, j13);
  }
};
template <int DIR>
struct DftScaled<4, DIR, 10> {  // c1 and c3 owe h
  static __device__ __forceinline__ void run(float2 (&a)[4]) {
    const float2 s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
    const float2 u = cadd(a[1], a[3]), v = csub(a[1], a[3]);
    const float2 jv = cmul_i(v, float(DIR));
    a[0] = cfma(kH, u, s02);
    a[2] = cfma(-kH, u, s02);
    a[1] = cfma(kH, jv, d02);
    a[3] = cfma(-kH, jv, d02);
  }
};

// DFT of P points of the inputs s[n] a[n] (real scales, e.g. a sampling
// mask): radix 4 folds the scales into fused multiply-adds.
template <int P, int DIR>
struct DftInScaled {
  static __device__ __forceinline__ void run(float2 (&a)[P], const float (&s)[P]) {
#pragma unroll
    for (int n = 0; n < P; ++n) a[n] = cscale(a[n], s[n]);
    Dft<P, DIR>::run(a);
  }
};
template <int DIR>
struct DftInScaled<4, DIR> {
  static __device__ __forceinline__ void run(float2 (&a)[4], const float (&s)[4]) {
    const float2 t0 = cscale(a[0], s[0]), t1 = cscale(a[1], s[1]);
    const float2 s02 = cfma(s[2], a[2], t0), d02 = cfma(-s[2], a[2], t0);
    const float2 s13 = cfma(s[3], a[3], t1), d13 = cfma(-s[3], a[3], t1);
    const float2 j13 = cmul_i(d13, float(DIR));
    a[0] = cadd(s02, s13);
    a[2] = csub(s02, s13);
    a[1] = cadd(d02, j13);
    a[3] = csub(d02, j13);
  }
};

template <int R, int DIR>
struct Dft {
  // composite: n = Q n1 + n2, k = k1 + P k2; the inter-level twiddles that
  // are odd multiples of 45 degrees leave their factor h to the second level
  static __device__ __forceinline__ void run(float2 (&a)[R]) {
    constexpr int P = Split<R>::P, Q = Split<R>::Q;
    float2 Y[Q][P];
#pragma unroll
    for (int n2 = 0; n2 < Q; ++n2) {
      float2 b[P];
#pragma unroll
      for (int n1 = 0; n1 < P; ++n1) b[n1] = a[Q * n1 + n2];
      Dft<P, DIR>::run(b);
#pragma unroll
      for (int k1 = 0; k1 < P; ++k1) Y[n2][k1] = b[k1];
    }
    second_level(Y, a);
  }
  // the DFT of s[n] a[n] (real per-input scales)
  static __device__ __forceinline__ void run_in_scaled(float2 (&a)[R], const float (&sc)[R]) {
    constexpr int P = Split<R>::P, Q = Split<R>::Q;
    float2 Y[Q][P];
#pragma unroll
    for (int n2 = 0; n2 < Q; ++n2) {
      float2 b[P];
      float sb[P];
#pragma unroll
      for (int n1 = 0; n1 < P; ++n1) {
        b[n1] = a[Q * n1 + n2];
        sb[n1] = sc[Q * n1 + n2];
      }
      DftInScaled<P, DIR>::run(b, sb);
#pragma unroll
      for (int k1 = 0; k1 < P; ++k1) Y[n2][k1] = b[k1];
    }
    second_level(Y, a);
  }
  static __device__ __forceinline__ void second_level(float2 (&Y)[Split<R>::Q][Split<R>::P], float2 (&a)[R]) {
    constexpr int P = Split<R>::P, Q = Split<R>::Q;
    static_for<0, P>([&](auto k1c) {
      constexpr int k1 = decltype(k1c)::value;
      float2 c[Q];
      static_for<0, Q>([&](auto n2c) {
        constexpr int n2 = decltype(n2c)::value;
        if constexpr (Tw45<R, n2 * k1>::value)
          c[n2] = tw45_unscaled<R, n2 * k1, DIR>(Y[n2][k1]);
        else
          c[n2] = tw_mul<R, n2 * k1, DIR>(Y[n2][k1]);
      });
      DftScaled<Q, DIR, scaled_mask<R, Q, k1>()>::run(c);
#pragma unroll
      for (int k2 = 0; k2 < Q; ++k2) a[k1 + P * k2] = c[k2];
    });
  }
  template <int RR, int QQ, int K1>
  static constexpr int scaled_mask() {
    int m = 0;
    for (int n2 = 0; n2 < QQ; ++n2) {
      const int k = ((n2 * K1) % RR + RR) % RR;
      if (k != 0 && (8 * k) % RR == 0 && (((8 * k) / RR) & 1) == 1) m |= 1 << n2;
    }
    return m;
  }
};

template <int DIR>
struct Dft<1, DIR> {
  static __device__ __forceinline__ void run(float2 (&)[1]) {}
};

template <int DIR>
struct Dft<2, DIR> {
  static __device__ __forceinline__ void run(float2 (&a)[2]) {
    const float2 t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  }
};

template <int DIR>
struct Dft<4, DIR> {
  static __device__ __forceinline__ void run(float2 (&a)[4]) {
    const float2 s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
    const float2 s13 = cadd(a[1], a[3]), d13 = csub(a[1], a[3]);
    const float2 j13 = cmul_i(d13, float(DIR));
    a[0] = cadd(s02, s13);
    a[2] = csub(s02, s13);
    a[1] = cadd(d02, j13);
    a[3] = csub(d02, j13);
  }
};

// Odd prime radix by symmetric pairs:
// X_k = a_0 + sum_n s_n cos(2 pi n k / R) + i DIR sum_n d_n sin(2 pi n k / R)
// with s_n = a_n + a_{R-n}, d_n = a_n - a_{R-n}; X_{R-k} flips the sine part.
template <int R, int DIR>
struct DftOdd {
  static __device__ __forceinline__ void run(float2 (&a)[R]) {
    constexpr int H = (R - 1) / 2;
    float2 s[H], d[H];
    float2 sum = a[0];
#pragma unroll
    for (int n = 1; n <= H; ++n) {
      s[n - 1] = cadd(a[n], a[R - n]);
      d[n - 1] = csub(a[n], a[R - n]);
      sum = cadd(sum, s[n - 1]);
    }
    float2 out[R];
    out[0] = sum;
    static_for<1, H + 1>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      float2 re = a[0], im = make_float2(0.f, 0.f);
      static_for<1, H + 1>([&](auto nc) {
        constexpr int n = decltype(nc)::value;
        constexpr float c = TwC<R, n * k, 1>::re;
        constexpr float sn = TwC<R, n * k, 1>::im;  // sin(2 pi n k / R)
        re = make_float2(re.x + c * s[n - 1].x, re.y + c * s[n - 1].y);
        im = make_float2(im.x + sn * d[n - 1].x, im.y + sn * d[n - 1].y);
      });
      const float2 jim = cmul_i(im, float(DIR));
      out[k] = cadd(re, jim);
      out[R - k] = csub(re, jim);
    });
#pragma unroll
    for (int k = 0; k < R; ++k) a[k] = out[k];
  }
};
template <int DIR> struct Dft<3, DIR> : DftOdd<3, DIR> {};
template <int DIR> struct Dft<5, DIR> : DftOdd<5, DIR> {};
template <int DIR> struct Dft<7, DIR> : DftOdd<7, DIR> {};

// ---------------------------------------------------------------- plans

template <int... Rs>
struct Radices {};

template <int N>
struct Plan;
template <> struct Plan<64> { static constexpr int NT = 8; using R = Radices<8, 8>; };
template <> struct Plan<128> { static constexpr int NT = 8; using R = Radices<16, 8>; };
template <> struct Plan<192> { static constexpr int NT = 16; using R = Radices<12, 4, 4>; };
template <> struct Plan<224> { static constexpr int NT = 8; using R = Radices<28, 4, 2>; };
template <> struct Plan<256> { static constexpr int NT = 16; using R = Radices<16, 16>; };
template <> struct Plan<320> { static constexpr int NT = 16; using R = Radices<20, 4, 4>; };
template <> struct Plan<512> { static constexpr int NT = 64; using R = Radices<8, 8, 8>; };
template <> struct Plan<1024> { static constexpr int NT = 64; using R = Radices<16, 16, 4>; };

// Offsets of each length's table inside the packed twiddle buffer
// (tw[k] = exp(-2 pi i k / N), k < N).
__host__ __device__ constexpr int tw_offset(int N) {
  return N == 64 ? 0 : N == 128 ? 64 : N == 192 ? 192 : N == 224 ? 384 : N == 256 ? 608
       : N == 320 ? 864 : N == 512 ? 1184 : N == 1024 ? 1696 : -1;
}
constexpr int kTwiddleTotal = 2720;
constexpr int kSupportedSizes[] = {64, 128, 192, 224, 256, 320, 512, 1024};
// X-macro over the same lengths (one kernel instance per length in the launchers)
#define PICS_FFT_SIZES(X) X(64) X(128) X(192) X(224) X(256) X(320) X(512) X(1024)

// LDS layouts: Lay::addr(idx, seq) gives the slot of element idx of sequence
// seq.  Column tiles keep T sequences side by side (row-major like global
// memory); row tiles keep each sequence contiguous with one pad slot per 16.
// Tiles narrower than 16 columns pad 4 slots per 16 elements to spread the
// first exchange's stores over the banks.
template <int T>
struct ColLay {
  static constexpr int pad = T < 16 ? 4 : 0;
  template <int M>
  static constexpr int size = M * T + ((M + 15) / 16) * pad;
  static __device__ __forceinline__ int addr(int idx, int seq) { return idx * T + seq + (idx >> 4) * pad; }
};
template <int N>
struct RowLay {
  static constexpr int stride = N + N / 16 + 4;
  static __device__ __forceinline__ int addr(int idx, int seq) { return seq * stride + idx + (idx >> 4); }
};

// DUAL: exchanges alternate between lds and lds_next and the barrier after
// each exchange's reads is left out (the next exchange writes the other
// buffer; the one after that is ordered by the next exchange's barrier).
// SCALE_IN: the first stage transforms s[e] v[e] (the inputs scaled by the
// real factors `in_scale`, e.g. a sampling mask); later stages ignore it.
template <int N, int NT, int DIR, int Ns, class Lay, bool DUAL, bool SCALE_IN, int R, int... Rest>
__device__ __forceinline__ void fft_stages(float2 (&v)[N / NT], int t, float2* lds, float2* lds_next, int seq,
                                           const float2* __restrict__ tw, const float (&in_scale)[N / NT]) {
  constexpr int E = N / NT;
  constexpr int Q = E / R;
  static_assert(E % R == 0, "radix must divide the elements per thread");
  constexpr bool LAST = sizeof...(Rest) == 0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int b = t + NT * q;
    float2 u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[q + r * Q];
    const int bm = b % Ns;
    if constexpr (Ns > 1) {
      constexpr int step = N / (Ns * R);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = tw[bm * r * step];
        if constexpr (DIR > 0) w.y = -w.y;
        u[r] = cmul(u[r], w);
      }
    }
    if constexpr (SCALE_IN && Ns == 1) {
      float us[R];
#pragma unroll
      for (int r = 0; r < R; ++r) us[r] = in_scale[q + r * Q];
      if constexpr (R >= 8)
        Dft<R, DIR>::run_in_scaled(u, us);
      else
        DftInScaled<R, DIR>::run(u, us);
    } else {
      Dft<R, DIR>::run(u);
    }
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[q + r * Q] = u[r];
    } else {
      const int base = (b / Ns) * Ns * R + bm;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[Lay::addr(base + r * Ns, seq)] = u[r];
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = lds[Lay::addr(t + NT * e, seq)];
    if constexpr (DUAL) {
      fft_stages<N, NT, DIR, Ns * R, Lay, DUAL, SCALE_IN, Rest...>(v, t, lds_next, lds, seq, tw, in_scale);
    } else {
      __syncthreads();
      fft_stages<N, NT, DIR, Ns * R, Lay, DUAL, SCALE_IN, Rest...>(v, t, lds, lds, seq, tw, in_scale);
    }
  }
}

template <class R>
struct RadixCount;
template <int... Rs>
struct RadixCount<Radices<Rs...>> { static constexpr int value = sizeof...(Rs); };
// LDS exchanges of one transform of length N (stages - 1)
template <int N>
constexpr int kExchanges = RadixCount<typename Plan<N>::R>::value - 1;

template <int N, int DIR, class Lay, bool DUAL, bool SCALE_IN = false, int... Rs>
__device__ __forceinline__ void fft_run(Radices<Rs...>, float2 (&v)[N / Plan<N>::NT], int t, float2* lds,
                                        float2* lds_next, int seq, const float2* __restrict__ tw,
                                        const float (&in_scale)[N / Plan<N>::NT]) {
  fft_stages<N, Plan<N>::NT, DIR, 1, Lay, DUAL, SCALE_IN, Rs...>(v, t, lds, lds_next, seq, tw, in_scale);
}
template <int N, int DIR, class Lay, bool DUAL, int... Rs>
__device__ __forceinline__ void fft_run(Radices<Rs...> r, float2 (&v)[N / Plan<N>::NT], int t, float2* lds,
                                        float2* lds_next, int seq, const float2* __restrict__ tw) {
  const float none[N / Plan<N>::NT] = {};
  fft_run<N, DIR, Lay, DUAL, false>(r, v, t, lds, lds_next, seq, tw, none);
}

// In-place transform of the cyclic registers.  Every thread of the block must
// call it (it contains barriers).  `tw` points at this length's table.  The
// LDS buffer may be reused as soon as it returns.
template <int N, int DIR, class Lay>
__device__ __forceinline__ void fft(float2 (&v)[N / Plan<N>::NT], int t, float2* lds, int seq,
                                    const float2* __restrict__ tw) {
  fft_run<N, DIR, Lay, false>(typename Plan<N>::R{}, v, t, lds, lds, seq, tw);
}

// Same transform with its exchanges alternating between two LDS buffers,
// first `lds_a`.  A caller chaining transforms keeps the alternation going
// (the next transform starts on the buffer after the last one used: b when
// kExchanges<N> is odd); the last exchange's buffer must not be written
// before another barrier.
template <int N, int DIR, class Lay>
__device__ __forceinline__ void fft_dual(float2 (&v)[N / Plan<N>::NT], int t, float2* lds_a, float2* lds_b,
                                         int seq, const float2* __restrict__ tw) {
  fft_run<N, DIR, Lay, true>(typename Plan<N>::R{}, v, t, lds_a, lds_b, seq, tw);
}

// The transform of in_scale[e] v[e]: the real per-element factors (a sampling
// mask with its normalisation) are folded into the first stage's additions.
// Single-buffer (DUAL = false) or dual-buffer exchanges as fft / fft_dual.
template <int N, int DIR, class Lay, bool DUAL>
__device__ __forceinline__ void fft_in_scaled(float2 (&v)[N / Plan<N>::NT], const float (&in_scale)[N / Plan<N>::NT],
                                              int t, float2* lds_a, float2* lds_b, int seq,
                                              const float2* __restrict__ tw) {
  fft_run<N, DIR, Lay, DUAL, true>(typename Plan<N>::R{}, v, t, lds_a, DUAL ? lds_b : lds_a, seq, tw, in_scale);
}

}  // namespace pics

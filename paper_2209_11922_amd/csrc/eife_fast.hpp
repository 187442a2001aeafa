// Fast sine-transform passes for power-of-two lines (N in {64, 128, 256, 512}).
//
// Same arithmetic as the generic passes (odd extension of two packed lines,
// FFT of length L = 2N, Section 4), organised for gfx950:
//   * one line pair per wavefront slice of LP = L / E lanes, E complex values
//     per lane, compile-time radix-8/16 Stockham stages whose exchanges stay
//     inside the wavefront (no block barrier inside an FFT);
//   * the block stages a tile of lines in LDS with coalesced global loads and
//     stores (row segments of C columns for strided axes, whole rows for x);
//   * the first FFT stage reads the odd extension straight from the tile, the
//     last stage leaves the outputs in registers.
#pragma once

#include "eife_kernels.hpp"

namespace eife {
namespace fast {

template <typename T, int R>
struct DftN {
  static __device__ __forceinline__ void run(Cx<T>* v) { Dft<T, R>::run(v); }
};

template <typename T>
struct DftN<T, 8> {
  static __device__ __forceinline__ void run(Cx<T>* x) {
    const T r = T(0.70710678118654752440);
    Cx<T> a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[q] = cadd(x[q], x[q + 4]);
      b[q] = csub(x[q], x[q + 4]);
    }
    b[1] = Cx<T>{(b[1].re + b[1].im) * r, (b[1].im - b[1].re) * r};
    b[2] = Cx<T>{b[2].im, -b[2].re};
    b[3] = Cx<T>{(b[3].im - b[3].re) * r, -(b[3].re + b[3].im) * r};
    Dft<T, 4>::run(a);
    Dft<T, 4>::run(b);
    x[0] = a[0];
    x[2] = a[1];
    x[4] = a[2];
    x[6] = a[3];
    x[1] = b[0];
    x[3] = b[1];
    x[5] = b[2];
    x[7] = b[3];
  }
};

template <typename T>
struct DftN<T, 16> {
  static __device__ __forceinline__ void run(Cx<T>* x) {
    // cos / sin of 2 pi m / 16, m = 0..9
    const T C[10] = {T(1.0), T(0.92387953251128675613), T(0.70710678118654752440), T(0.38268343236508977173),
                     T(0.0), T(-0.38268343236508977173), T(-0.70710678118654752440), T(-0.92387953251128675613),
                     T(-1.0), T(-0.92387953251128675613)};
    const T S[10] = {T(0.0), T(0.38268343236508977173), T(0.70710678118654752440), T(0.92387953251128675613),
                     T(1.0), T(0.92387953251128675613), T(0.70710678118654752440), T(0.38268343236508977173),
                     T(0.0), T(-0.38268343236508977173)};
    Cx<T> y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      Cx<T> t[4] = {x[n2], x[4 + n2], x[8 + n2], x[12 + n2]};
      Dft<T, 4>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) {
        const int m = n2 * k1;  // twiddle exp(-2 pi i m / 16)
        if (m == 0)
          y[n2][k1] = t[k1];
        else
          y[n2][k1] = cmul(t[k1], Cx<T>{C[m], -S[m]});
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      Cx<T> t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
      Dft<T, 4>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) x[k1 + 4 * k2] = t[k2];
    }
  }
};

// Padded index in a pair's exchange buffer (one pad slot every 8 entries).
__device__ __forceinline__ int xpad(int i) { return i + (i >> 3); }

template <int L>
struct FftShape {
  static constexpr int E = (L <= 512) ? 8 : 16;  // complex values per lane
  static constexpr int LP = L / E;                // lanes per line pair
  static constexpr int R2 = L / (E * E);          // radix of the third stage
  // pair region: padded exchange buffer, stride = 2 (mod 64) complex so that
  // the column-tile accesses (16 pairs x rows) are free of LDS bank conflicts
  static constexpr int BUF = ((L + L / 8 + 63) / 64) * 64 + 2;
  static constexpr int NB2 = E / R2;              // third-stage butterflies per lane
  static_assert(LP <= 64, "a line pair must fit in one wavefront");
  static_assert(R2 >= 2 && R2 <= E, "unsupported FFT length");
};

// Occupancy hint (waves per SIMD) of the pass kernels: 4 keeps two 8-wave
// blocks per CU for FP32 lines up to 512 points; longer, double or
// three-subsequence lines need more registers than that leaves.
template <typename T, int L>
struct MinWaves {
  static constexpr int value = (L >= 1024 || sizeof(T) == 8 || (L & (L - 1)) != 0) ? 2 : 4;
};

// The twiddle factors one lane needs, loaded once per kernel.  FP32 lanes of
// lines up to 512 points keep every factor in registers; FP64 lanes and FP32
// lanes of 1024-point lines keep the two generators only (FP64 512: 16
// registers instead of 56) and form the powers for each stage as it starts
// (balanced products, a few ulps), so that these passes fit more waves.
template <typename T, int L>
struct LaneTw {
  static constexpr int E = FftShape<L>::E;
  static constexpr int R2 = FftShape<L>::R2;
  static constexpr int NB2 = FftShape<L>::NB2;
  static constexpr int LP = FftShape<L>::LP;
  static constexpr bool POW = sizeof(T) == 8 || L >= 1024;
  static constexpr int S1 = POW ? 1 : E;
  static constexpr int S2 = POW ? 1 : R2;
  Cx<T> s1[S1 > 1 ? S1 : 2];  // stage 2 (Ns = E): W_L^{q k (L / E^2)}, k = lane mod E (POW: q = 1 only)
  Cx<T> s2[NB2][S2 > 1 ? S2 : 2];  // stage 3 (Ns = E^2): W_L^{q j}, j = lane + LP b (POW: q = 1 only)
  // tw[i] = exp(-2 pi i i / (L * stride)): the table of a line stride times as long
  __device__ __forceinline__ void load(const Cx<T>* __restrict__ tw, int lane, int stride = 1) {
    const int k = lane & (E - 1);
#pragma unroll
    for (int q = 1; q < (POW ? 2 : E); ++q) s1[q] = tw[stride * (q * k) * (L / (E * E))];
#pragma unroll
    for (int b = 0; b < NB2; ++b) {
      const int j = lane + LP * b;
#pragma unroll
      for (int q = 1; q < (POW ? 2 : R2); ++q) s2[b][q] = tw[stride * q * j];
    }
  }
};

// Powers p[q] = g^q, q = 1 .. R - 1, by balanced products.
template <typename T, int R>
__device__ __forceinline__ void tw_powers(Cx<T> g, Cx<T> (&p)[R]) {
  p[1] = g;
#pragma unroll
  for (int q = 2; q < R; ++q) p[q] = (q & 1) ? cmul(p[q - 1], g) : cmul(p[q / 2], p[q / 2]);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One Stockham stage of radix R on the pair owned by this lane group.
// `in(b, q)` yields input q of butterfly b (stage input index
// j + (L/R) q, j = lane + LP b); `tw(b, q)` its twiddle.  Unless LAST, the
// outputs are written to buf, else they stay in v
// (v[b*R+q] = output lane + LP*b + q*(L/R)).
// Padded indices: xpad(B + 8t) = xpad(B) + 9t, so every buffer access is a
// per-lane base plus a compile-time offset.
template <typename T, int L, int R, int Ns, bool LAST, typename In, typename Tw>
__device__ __forceinline__ void wstage(Cx<T> (&v)[FftShape<L>::E], In in, Tw twf, Cx<T>* buf, int lane) {
  constexpr int E = FftShape<L>::E;
  constexpr int LP = FftShape<L>::LP;
  constexpr int NB = E / R;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int q = 0; q < R; ++q) v[b * R + q] = in(b, q);
    if constexpr (Ns > 1) {
#pragma unroll
      for (int q = 1; q < R; ++q) v[b * R + q] = cmul(v[b * R + q], twf(b, q));
    }
    DftN<T, R>::run(&v[b * R]);
  }
  if constexpr (!LAST) {
    if constexpr (Ns == 1) {
      // base = R j: xpad(R j + q) = R j + (R j >> 3) + q + (q >> 3) (R multiple of 8)
      static_assert(R % 8 == 0, "first stage radix must be a multiple of 8");
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = lane + LP * b;
        Cx<T>* o = buf + R * j + ((R * j) >> 3);
#pragma unroll
        for (int q = 0; q < R; ++q) o[q + (q >> 3)] = v[b * R + q];
      }
    } else {
      static_assert(Ns % 8 == 0, "stride of later stages must be a multiple of 8");
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = lane + LP * b;
        const int k = j & (Ns - 1);
        const int base = (j - k) * R + k;
        Cx<T>* o = buf + xpad(base);
#pragma unroll
        for (int q = 0; q < R; ++q) o[q * Ns + (q * Ns) / 8] = v[b * R + q];
      }
    }
  }
}

// Stages 2 and 3 of a length-L FFT whose first stage has been written to buf.
template <typename T, int L>
__device__ __forceinline__ void fft_tail(Cx<T> (&v)[FftShape<L>::E], Cx<T>* buf, int lane, const LaneTw<T, L>& tw) {
  constexpr int E = FftShape<L>::E;
  constexpr int LP = FftShape<L>::LP;
  constexpr int R2 = FftShape<L>::R2;
  // input j + (L/R) q sits at xpad(j) + (L/R) q * 9/8
  const Cx<T>* rb = buf + xpad(lane);
  auto in1 = [&](int, int q) -> Cx<T> { return rb[(L / E) * q + (L / E) * q / 8]; };
  auto in2 = [&](int b, int q) -> Cx<T> {
    return rb[LP * b + (LP * b) / 8 + (L / R2) * q + (L / R2) * q / 8];
  };
  if constexpr (LaneTw<T, L>::POW) {
    constexpr int NB2 = FftShape<L>::NB2;
    Cx<T> p1[E];
    tw_powers<T, E>(tw.s1[1], p1);
    auto tw1 = [&](int, int q) -> Cx<T> { return p1[q]; };
    wstage<T, L, E, E, false>(v, in1, tw1, buf, lane);
    wave_sync();
    Cx<T> p2[NB2][R2];
#pragma unroll
    for (int b = 0; b < NB2; ++b) tw_powers<T, R2>(tw.s2[b][1], p2[b]);
    auto tw2 = [&](int b, int q) -> Cx<T> { return p2[b][q]; };
    wstage<T, L, R2, E * E, true>(v, in2, tw2, buf, lane);
  } else {
    auto tw1 = [&](int, int q) -> Cx<T> { return tw.s1[q]; };
    auto tw2 = [&](int b, int q) -> Cx<T> { return tw.s2[b][q]; };
    wstage<T, L, E, E, false>(v, in1, tw1, buf, lane);
    wave_sync();
    wstage<T, L, R2, E * E, true>(v, in2, tw2, buf, lane);
  }
}

// First stage of a length-L FFT on the inputs already in v (v[q] = input lane + LP q).
template <typename T, int L>
__device__ __forceinline__ void fft_head(Cx<T> (&v)[FftShape<L>::E], Cx<T>* buf, int lane) {
  constexpr int E = FftShape<L>::E;
  auto inr = [&](int, int q) -> Cx<T> { return v[q]; };
  auto tw0 = [&](int, int) -> Cx<T> { return Cx<T>{T(1), T(0)}; };
  wstage<T, L, E, 1, false>(v, inr, tw0, buf, lane);
}

// Forward FFT of length L of the odd extension of the pair whose node values
// sit at node[0 .. N-2].  On return v holds the outputs (see wstage with LAST).
template <typename T, int L>
__device__ __forceinline__ void odd_fft(Cx<T> (&v)[FftShape<L>::E], const Cx<T>* node, Cx<T>* buf, int lane,
                                        const LaneTw<T, L>& tw) {
  constexpr int E = FftShape<L>::E;
  constexpr int LP = FftShape<L>::LP;
  constexpr int N = L / 2;
  // stage 0: input m = lane + LP q; q < E/2 <=> m < N
  const Cx<T>* lo = node + (lane - 1);          // node[m - 1]
  const Cx<T>* hi = node + (2 * N - 1 - lane);  // node[2N - m - 1] = hi[-LP q]
#pragma unroll
  for (int q = 0; q < E; ++q) {
    if (q < E / 2) {
      v[q] = (q == 0 && lane == 0) ? Cx<T>{T(0), T(0)} : lo[LP * q];
    } else if (q == E / 2 && lane == 0) {
      v[q] = Cx<T>{T(0), T(0)};
    } else {
      const Cx<T> c = hi[-LP * q];
      v[q] = Cx<T>{-c.re, -c.im};
    }
  }
  fft_head<T, L>(v, buf, lane);
  wave_sync();
  fft_tail<T, L>(v, buf, lane, tw);
  wave_sync();  // buf may be rewritten by the next transform of this pair
}

// Visit the outputs k in [1, N-1] held by this lane: f(k, Z_k); k = lane + c
// with c a compile-time offset for every entry.
template <typename T, int L, typename F>
__device__ __forceinline__ void for_outputs(const Cx<T> (&v)[FftShape<L>::E], int lane, F f) {
  constexpr int E = FftShape<L>::E;
  constexpr int LP = FftShape<L>::LP;
  constexpr int R2 = FftShape<L>::R2;
  constexpr int NB = E / R2;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int q = 0; q < R2 / 2; ++q) {
      const int k = lane + LP * b + q * (L / R2);
      if (k >= 1) f(k, v[b * R2 + q]);
    }
  }
}

// ---------------------------------------------------------------------------
// Line<T, L>: the transform of one line pair of FFT length L = 2N, for L a
// power of two (one wave-local FFT) or L = 3M with M a power of two (the
// odd extension split into its three stride-3 subsequences, three M-point
// wave FFTs, then a radix-3 combination:
//   Z_{k'+jM} = F0_{k'} + w^j W_L^{k'} F1_{k'} + w^{2j} W_L^{2k'} F2_{k'},  w = exp(-2 pi i/3)).
// Interface: LP (lanes per pair), BUF (LDS region per pair), Regs, Tw,
// transform(regs, node, region, lane, tw, twL), outputs(regs, lane, twL, f).
template <int L>
struct IsPow2 {
  static constexpr bool value = (L & (L - 1)) == 0;
};

template <typename T, int L, bool P2 = IsPow2<L>::value>
struct Line;

template <typename T, int L>
struct Line<T, L, true> {
  static constexpr int LP = FftShape<L>::LP;
  static constexpr int BUF = FftShape<L>::BUF;
  struct Regs {
    Cx<T> v[FftShape<L>::E];
  };
  struct Tw {
    LaneTw<T, L> t;
    __device__ __forceinline__ void load(const Cx<T>* __restrict__ tw, int lane) { t.load(tw, lane, 1); }
  };
  static __device__ __forceinline__ void transform(Regs& r, const Cx<T>* node, Cx<T>* region, int lane, const Tw& tw,
                                                   const Cx<T>* __restrict__) {
    odd_fft<T, L>(r.v, node, region, lane, tw.t);
  }
  template <typename F>
  static __device__ __forceinline__ void outputs(const Regs& r, int lane, const Cx<T>* __restrict__, F f) {
    for_outputs<T, L>(r.v, lane, f);
  }
};

template <typename T, int L>
struct Line<T, L, false> {
  static constexpr int M = L / 3;
  static_assert(3 * M == L && IsPow2<M>::value, "line length must be 2^k or 3 * 2^k");
  static constexpr int E = FftShape<M>::E;
  static constexpr int LP = FftShape<M>::LP;
  static constexpr int R2 = FftShape<M>::R2;
  static constexpr int SUB = M + M / 8;  // exchange buffer of one sub-transform (multiple of 8)
  static constexpr int BUF = ((3 * SUB + 63) / 64) * 64 + 2;
  struct Regs {
    Cx<T> v[3][E];
  };
  struct Tw {
    LaneTw<T, M> t;
    __device__ __forceinline__ void load(const Cx<T>* __restrict__ tw, int lane) { t.load(tw, lane, 3); }
  };
  static __device__ __forceinline__ void transform(Regs& r, const Cx<T>* node, Cx<T>* region, int lane, const Tw& tw,
                                                   const Cx<T>* __restrict__) {
    constexpr int N = L / 2;
    // every node value is read before the exchange buffers (which overlay the
    // nodes) are written
#pragma unroll
    for (int s = 0; s < 3; ++s) {
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int p = 3 * (lane + LP * q) + s;  // index in the odd extension
        Cx<T> val = Cx<T>{T(0), T(0)};
        if (p != 0 && p != N) {
          if (p < N) {
            val = node[p - 1];
          } else {
            const Cx<T> c = node[L - p - 1];
            val = Cx<T>{-c.re, -c.im};
          }
        }
        r.v[s][q] = val;
      }
    }
    wave_sync();
#pragma unroll
    for (int s = 0; s < 3; ++s) fft_head<T, M>(r.v[s], region + s * SUB, lane);
    wave_sync();
#pragma unroll
    for (int s = 0; s < 3; ++s) fft_tail<T, M>(r.v[s], region + s * SUB, lane, tw.t);
    wave_sync();
  }
  template <typename F>
  static __device__ __forceinline__ void outputs(const Regs& r, int lane, const Cx<T>* __restrict__ twL, F f) {
    constexpr int NB = E / R2;
    const T h = T(0.86602540378443864676);  // sqrt(3)/2
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int q = 0; q < R2; ++q) {
        const int kp = lane + LP * b + q * (M / R2);  // output of the sub-transforms, 0 <= kp < M
        const Cx<T> f0 = r.v[0][b * R2 + q];
        const Cx<T> t1 = cmul(r.v[1][b * R2 + q], twL[kp]);
        const Cx<T> t2 = cmul(r.v[2][b * R2 + q], twL[2 * kp]);
        const Cx<T> sum = cadd(t1, t2);
        if (kp >= 1) f(kp, cadd(f0, sum));
        if (kp < M / 2) {
          const Cx<T> d = csub(t1, t2);
          // f0 + w t1 + w^2 t2 = f0 - sum/2 - i (sqrt(3)/2) d
          f(M + kp, Cx<T>{f0.re - T(0.5) * sum.re + h * d.im, f0.im - T(0.5) * sum.im - h * d.re});
        }
      }
    }
  }
};

// ---------------------------------------------------------------------------
// Each line pair owns one LDS region of FftShape<L>::BUF complex entries.  Its
// first N - 1 entries hold the pair's node values (the "tile"); the whole
// region doubles as the pair's FFT exchange buffer, which is safe because
// stage 1 has read every node value before it writes the region and only
// the pair's own wavefront slice touches it between block barriers.

// Reaction kinds that get their own code path (everything else is generic).
enum { RK_GENERIC = 0, RK_AC = 1 };

template <typename T, int RK>
__device__ __forceinline__ T reaction_k(const Forcing& F, T u, int ix, int iy, int iz) {
  if (RK == RK_AC) return u - u * u * u;
  return reaction<T, false>(F, u, ix, iy, iz);
}

// ---------------------------------------------------------------------------
// Row passes (x lines, contiguous).  Block = PB line pairs = 2 PB rows; each
// wavefront slice loads, transforms and stores its own pair, so the pass
// needs no block barrier.
template <typename T, int L, int PB, int MODE, int RK, bool BAT>
__global__ void __launch_bounds__((PB * Line<T, L>::LP), (MinWaves<T, L>::value)) row_fast(const T* src, T* dst, T* dst2, RowGeom g,
                                                                     const Cx<T>* __restrict__ tw, Forcing F,
                                                                     const RowInst<T>* __restrict__ insts) {
  if constexpr (BAT) row_inst_ptrs<T, MODE>(insts, src, dst, dst2, F);
  using Ln = Line<T, L>;
  constexpr int N = L / 2;
  constexpr int n = N - 1;
  constexpr int LP = Ln::LP;
  constexpr int BUF = Ln::BUF;
  constexpr int RIT = (n + LP - 1) / LP;
  __shared__ Cx<T> lds[PB * BUF];
  const int tid = threadIdx.x;
  const int p = tid / LP;
  const int lane = tid - p * LP;
  const int ra = blockIdx.x * 2 * PB + 2 * p, rb = ra + 1;
  const bool hasa = ra < g.nrows, hasb = rb < g.nrows;
  const T scale = T(1.0 / sqrt(double(L)));
  typename Ln::Tw twl;
  twl.load(tw, lane);
  Cx<T>* my = lds + p * BUF;

  T va[RIT], vb[RIT];
  {
    const T* sa = src + int64_t(ra) * g.ld_src + lane;
    const T* sb = src + int64_t(rb) * g.ld_src + lane;
#pragma unroll
    for (int t = 0; t < RIT; ++t) {
      const bool in = lane + LP * t < n;
      va[t] = (in && hasa) ? sa[LP * t] : T(0);
      vb[t] = (in && hasb) ? sb[LP * t] : T(0);
    }
#pragma unroll
    for (int t = 0; t < RIT; ++t)
      if (lane + LP * t < n) my[lane + LP * t] = Cx<T>{va[t], vb[t]};
  }
  wave_sync();

  typename Ln::Regs v;
  Ln::transform(v, my, my, lane, twl, tw);

  if (MODE == ROW_FWD_PHYS) {
    // dst2 = S_x u; then the reaction of the loaded nodal values, forward
    Ln::outputs(v, lane, tw, [&](int k, Cx<T> Z) { my[k - 1] = Cx<T>{-Z.im * scale, Z.re * scale}; });
    wave_sync();
    {
      T* ha = dst2 + int64_t(ra) * g.ld_dst + lane;
      T* hb = dst2 + int64_t(rb) * g.ld_dst + lane;
      Cx<T> hv[RIT];
#pragma unroll
      for (int t = 0; t < RIT; ++t) hv[t] = my[lane + LP * t];
#pragma unroll
      for (int t = 0; t < RIT; ++t) {
        if (lane + LP * t < n) {
          if (hasa) ha[LP * t] = hv[t].re;
          if (hasb) hb[LP * t] = hv[t].im;
        }
      }
    }
    wave_sync();
    const int iya = ra % g.ny, iza = ra / g.ny;
    const int iyb = rb % g.ny, izb = rb / g.ny;
#pragma unroll
    for (int t = 0; t < RIT; ++t) {
      const int m = lane + LP * t;
      if (m < n)
        my[m] = Cx<T>{reaction_k<T, RK>(F, va[t], m, iya, iza), reaction_k<T, RK>(F, vb[t], m, iyb, izb)};
    }
    wave_sync();
    Ln::transform(v, my, my, lane, twl, tw);
  }

  if (MODE == ROW_PHYS) {
    const int iya = ra % g.ny, iza = ra / g.ny;
    const int iyb = rb % g.ny, izb = rb / g.ny;
    Ln::outputs(v, lane, tw, [&](int k, Cx<T> Z) {
      const T ua = -Z.im * scale, ub = Z.re * scale;
      const T fa = reaction_k<T, RK>(F, ua, k - 1, iya, iza);
      const T fb = reaction_k<T, RK>(F, ub, k - 1, iyb, izb);
      my[k - 1] = Cx<T>{fa, fb};
    });
    wave_sync();
    Ln::transform(v, my, my, lane, twl, tw);
  }
  Ln::outputs(v, lane, tw, [&](int k, Cx<T> Z) { my[k - 1] = Cx<T>{-Z.im * scale, Z.re * scale}; });
  wave_sync();
  T* da = dst + int64_t(ra) * g.ld_dst + lane;
  T* db = dst + int64_t(rb) * g.ld_dst + lane;
  T* da2 = dst2 + int64_t(ra) * g.ld_dst + lane;
  T* db2 = dst2 + int64_t(rb) * g.ld_dst + lane;
  Cx<T> outv[RIT];
#pragma unroll
  for (int t = 0; t < RIT; ++t) outv[t] = my[lane + LP * t];  // full b64 reads (slot n..N-1 is scratch)
  if constexpr (MODE == ROW_INV_CHG) {
    // the pair's sum of (u - u_n)^2: lane l takes its columns l, l + 64, ...
    // in order (row a, then row b), then a fixed butterfly over the lanes
    static_assert(LP == 64 && !BAT, "one wavefront per line pair");
    const T* ua = dst2 + int64_t(ra) * g.ld_dst + lane;
    const T* ub = dst2 + int64_t(rb) * g.ld_dst + lane;
    double sc = 0.0;
#pragma unroll
    for (int t = 0; t < RIT; ++t) {
      if (lane + LP * t < n) {
        if (hasa) {
          const double d = double(outv[t].re) - double(ua[LP * t]);
          sc = fma(d, d, sc);
        }
        if (hasb) {
          const double d = double(outv[t].im) - double(ub[LP * t]);
          sc = fma(d, d, sc);
        }
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sc += __shfl_xor(sc, o);
    if (lane == 0 && hasa) g.chg[ra >> 1] = sc;
  }
#pragma unroll
  for (int t = 0; t < RIT; ++t) {
    if (lane + LP * t < n) {
      if (hasa) da[LP * t] = outv[t].re;
      if (hasb) db[LP * t] = outv[t].im;
      if (MODE == ROW_FWD_USER) {
        if (hasa) da2[LP * t] = outv[t].re;
        if (hasb) db2[LP * t] = outv[t].im;
      }
    }
  }
}


template <int MODE>
__device__ __forceinline__ void diag_fast(const Sep& s, double D, double tau, double rtc2, double g, double h,
                                          double* out, double* nh) {
  const double G = g * s.w;
  const double rL = rcp64(D * s.lam);
  if (MODE == COL_ETD1) {
    const double un = fma(s.M, h - rL * G, h);  // h + M h - M rL G
    *out = un;
    *nh = un;
  } else if (MODE == COL_STAGE_A) {
    *out = fma(s.Mc, h - rL * G, h);
    const double a2 = s.Q * rL * rL * rtc2;  // tau phi_2 / c2
    *nh = fma(s.M, h, h) - fma(s.M, rL, a2) * G;
  } else {
    const double un = fma(s.Q * rL * rL * rtc2, G, h);
    *out = un;
    *nh = un;
  }
}

// ---------------------------------------------------------------------------
// Column passes (strided axis).  Block = PB pairs = C = 2 PB adjacent x-columns
// (C * sizeof(T) >= 128 bytes per row segment); each wavefront slice of LP
// lanes transforms PPW of the pairs one after the other.
// The three-stage modes carry more tables through the stage: 2 waves per SIMD
// (up to 256 registers per lane) keep them out of scratch.
template <typename T, int L, int MODE>
struct ColMinWaves {
  static constexpr int value = MODE >= COL_S3_1 ? 2 : MinWaves<T, L>::value;
};

// Block coordinates of a one-tile-per-block column pass.  The hardware hands
// linear block b (x fastest, then y, then z) to XCD b mod 8; tiles narrower
// than a 128-byte line share each line with the neighbouring tile, so for
// those the linear index is renumbered (b mod 8) * (nb / 8) + b / 8 (a
// bijection on the first 8 * (nb / 8) blocks) and the blocks of one XCD own
// a contiguous run of tiles: a shared line is fetched into one L2, not two.
template <typename T, int PB>
__device__ __forceinline__ void tile_coords(int& bx, int& by, int& bz) {
  bx = int(blockIdx.x);
  by = int(blockIdx.y);
  bz = int(blockIdx.z);
  if constexpr (2 * PB * int(sizeof(T)) < 128) {
    const int X = int(gridDim.x), Y = int(gridDim.y);
    const int nb = X * Y * int(gridDim.z);
    const int b = bx + X * (by + Y * bz);
    const int q = nb / 8;
    const int l = b < 8 * q ? (b % 8) * q + b / 8 : b;
    bx = l % X;
    by = (l / X) % Y;
    bz = l / (X * Y);
  }
}

template <typename T, int L, int PB, int PPW, int MODE, bool BAT>
__global__ void __launch_bounds__((PB / PPW * Line<T, L>::LP), (ColMinWaves<T, L, MODE>::value)) col_fast(T* W, T* H, ColGeom g, const Cx<T>* tw,
                                                                        Diag dg, const ColInst<T>* __restrict__ insts) {
  // per-instance tables of a batched launch are held in separate locals (a
  // modified copy of the Diag argument would live in private memory)
  AxisTab ta0 = dg.ax[0], ta1 = dg.ax[1], ta2 = dg.ax[2];
  double Dv = dg.D;
  int bx, by, bz;
  tile_coords<T, PB>(bx, by, bz);
  if constexpr (BAT) {
    if (insts) {
      const ColInst<T>& I = insts[bz];
      W = I.W;
      H = I.H;
      ta0 = I.ax[0];
      ta1 = I.ax[1];
      ta2 = I.ax[2];
      Dv = I.D;
    }
  }
  using Ln = Line<T, L>;
  constexpr int N = L / 2;
  constexpr int n = N - 1;
  constexpr int LP = Ln::LP;
  constexpr int BUF = Ln::BUF;
  constexpr int SLOTS = PB / PPW;
  constexpr int NT = SLOTS * LP;
  __shared__ Cx<T> lds[PB * BUF];
  const int tid = threadIdx.x;
  const int c0 = bx * 2 * PB;
  const int outer = by;
  const int64_t base = int64_t(outer) * g.ld_outer + c0;
  const T scale = T(1.0 / sqrt(double(L)));
  const int slot = tid / LP;
  const int lane = tid - slot * LP;

  // tile load: thread -> column pair q = tid % PB, rows m0 + MS it
  constexpr int MS = NT / PB;
  constexpr int CIT = (n + MS - 1) / MS;
  const int tq = tid % PB;
  const int m0 = tid / PB;
  const int ldl = int(g.ld_line);  // tile offsets stay below 2^31 elements
  const Cx<T>* gsrc = reinterpret_cast<const Cx<T>*>(W + base + m0 * ldl + 2 * tq);
  Cx<T>* ltile = lds + tq * BUF + m0;
  // narrow tiles (small grids, one wave per block): the stage's H values are
  // loaded together with the tile, so their latency overlaps the first FFT
  constexpr bool PREH = MODE != COL_PLAIN && PB <= 2;
  Cx<T> hpre[PREH ? CIT : 1];
  {
    Cx<T> tmp[CIT];
#pragma unroll
    for (int it = 0; it < CIT; ++it)
      if (m0 + MS * it < n) tmp[it] = gsrc[(MS * it * ldl) / 2];
    if constexpr (PREH) {
      const Cx<T>* hsrc = reinterpret_cast<const Cx<T>*>(H + base + m0 * ldl + 2 * tq);
#pragma unroll
      for (int it = 0; it < CIT; ++it)
        if (m0 + MS * it < n) hpre[it] = hsrc[(MS * it * ldl) / 2];
    }
#pragma unroll
    for (int it = 0; it < CIT; ++it)
      if (m0 + MS * it < n) ltile[MS * it] = mask_pad(tmp[it], c0 + 2 * tq, g.ncols);
  }
  __syncthreads();

  typename Ln::Regs v;
  {
    typename Ln::Tw twl;
    twl.load(tw, lane);
#pragma unroll 1
    for (int r = 0; r < PPW; ++r) {
      Cx<T>* my = lds + (slot + SLOTS * r) * BUF;
      Ln::transform(v, my, my, lane, twl, tw);
      Ln::outputs(v, lane, tw, [&](int k, Cx<T> Z) { my[k - 1] = Cx<T>{-Z.im * scale, Z.re * scale}; });
    }
  }

  if constexpr (MODE >= COL_S3_1) {
    // three-stage scheme (single grids only): the generic per-point stage on
    // the tile, reading H (and X) at the point
    static_assert(!BAT, "the three-stage passes take single grids");
    __syncthreads();
    // the column pair and the outer index are fixed per thread
    const S3K k3 = s3k_make(dg);
    Sep3 sxy[2];
    sep3_pair(dg, c0 + 2 * tq, g.last_is_z, outer, sxy);
#pragma unroll
    for (int it = 0; it < CIT; ++it) {
      const int m = m0 + MS * it;
      if (m < n) {
        const Cx<T> gv = ltile[MS * it];
        T outv[2];
        stage3_pair<T, MODE>(dg, k3, sxy, g.last_is_z, m, c0 + 2 * tq, base + int64_t(m) * g.ld_line + 2 * tq, H,
                             gv.re, gv.im, g.ncols, outv);
        ltile[MS * it] = Cx<T>{outv[0], outv[1]};
      }
    }
    __syncthreads();
    __asm__ volatile("" ::: "memory");
    typename Ln::Tw twl;
    twl.load(tw, lane);
#pragma unroll 1
    for (int r = 0; r < PPW; ++r) {
      Cx<T>* my = lds + (slot + SLOTS * r) * BUF;
      Ln::transform(v, my, my, lane, twl, tw);
      Ln::outputs(v, lane, tw, [&](int k, Cx<T> Z) { my[k - 1] = Cx<T>{-Z.im * scale, Z.re * scale}; });
    }
  } else if (MODE != COL_PLAIN) {
    __syncthreads();
    // diagonal stage over the tile: thread -> (row m, pair q), pair fixed per thread
    const double tau = dg.tau, D = Dv;
    const double rtc2 = 1.0 / (tau * dg.c2);
    const int q = tq;
    const int kx0 = c0 + 2 * q;
    Sep sxy[2];
    if (g.last_is_z) {
      const Sep sy = sep_load(ta1, outer);
      sxy[0] = sep_combine(sep_load(ta0, kx0), sy);
      sxy[1] = sep_combine(sep_load(ta0, kx0 + 1), sy);
    } else {
      const Sep sz = sep_load(ta2, 0);
      sxy[0] = sep_combine(sep_load(ta0, kx0), sz);
      sxy[1] = sep_combine(sep_load(ta0, kx0 + 1), sz);
    }
    const AxisTab line_tab = g.last_is_z ? ta2 : ta1;
    Cx<T>* hrow = reinterpret_cast<Cx<T>*>(H + base + m0 * ldl + 2 * q);
    constexpr int DIT = CIT;
    constexpr int BATCH = 4;
#pragma unroll
    for (int b0 = 0; b0 < DIT; b0 += BATCH) {
      Cx<T> hv[BATCH];
#pragma unroll
      for (int it = 0; it < BATCH; ++it) {
        const int m = m0 + (b0 + it) * MS;
        if (b0 + it < DIT && m < n) {
          if constexpr (PREH)
            hv[it] = hpre[b0 + it];
          else
            hv[it] = hrow[(MS * (b0 + it) * ldl) / 2];
        }
      }
#pragma unroll
      for (int it = 0; it < BATCH; ++it) {
        const int m = m0 + (b0 + it) * MS;
        if (b0 + it < DIT && m < n) {
          const Sep sl = sep_load(line_tab, m);
          const Cx<T> gv = ltile[MS * (b0 + it)];
          double o0, o1, n0, n1;
          diag_fast<MODE>(sep_combine(sxy[0], sl), D, tau, rtc2, double(gv.re), double(hv[it].re), &o0, &n0);
          diag_fast<MODE>(sep_combine(sxy[1], sl), D, tau, rtc2, double(gv.im), double(hv[it].im), &o1, &n1);
          hrow[(MS * (b0 + it) * ldl) / 2] = mask_pad(Cx<T>{T(n0), T(n1)}, kx0, g.ncols);
          ltile[MS * (b0 + it)] = Cx<T>{T(o0), T(o1)};
        }
      }
    }
    __syncthreads();
    __asm__ volatile("" ::: "memory");
    typename Ln::Tw twl;
    twl.load(tw, lane);
#pragma unroll 1
    for (int r = 0; r < PPW; ++r) {
      Cx<T>* my = lds + (slot + SLOTS * r) * BUF;
      Ln::transform(v, my, my, lane, twl, tw);
      Ln::outputs(v, lane, tw, [&](int k, Cx<T> Z) { my[k - 1] = Cx<T>{-Z.im * scale, Z.re * scale}; });
    }
  }
  __syncthreads();
  Cx<T>* gdst = reinterpret_cast<Cx<T>*>(W + base + m0 * ldl + 2 * tq);
#pragma unroll
  for (int it = 0; it < CIT; ++it)
    if (m0 + MS * it < n) gdst[(MS * it * ldl) / 2] = mask_pad(ltile[MS * it], c0 + 2 * tq, g.ncols);
}

// ---------------------------------------------------------------------------
// Persistent, software-pipelined plain column pass: each block walks tiles
// blockIdx.x, blockIdx.x + gridDim.x, ...; the next tile's loads are issued
// into registers before the current tile is transformed, so the memory
// latency hides behind the FFTs.  Tile t covers columns (t % ntx) * C ... and
// outer index t / ntx.
// First tile of a persistent column block (tiles t, t + gridDim.x, ...).  The
// hardware hands block b to XCD b mod 8; tiles narrower than a 128-byte line
// share each line with the neighbouring tile, so such blocks are renumbered
// (b mod 8) * (nb / 8) + b / 8 (a bijection on the first 8 * (nb / 8) blocks):
// the blocks of one XCD then own a contiguous run of tiles, and a shared line
// is fetched into one L2 instead of two.
template <typename T, int PB>
__device__ __forceinline__ int first_tile() {
  int b = int(blockIdx.x);
  if constexpr (2 * PB * int(sizeof(T)) < 128) {
    const int q = int(gridDim.x) / 8;
    if (b < 8 * q) b = (b % 8) * q + b / 8;
  }
  return b;
}

template <typename T, int L, int PB, int PPW>
__global__ void __launch_bounds__((PB / PPW * Line<T, L>::LP), (MinWaves<T, L>::value)) col_pipe(T* __restrict__ W, ColGeom g,
                                                                        const Cx<T>* tw, int ntx, int ntiles) {
  using Ln = Line<T, L>;
  constexpr int N = L / 2;
  constexpr int n = N - 1;
  constexpr int LP = Ln::LP;
  constexpr int BUF = Ln::BUF;
  constexpr int SLOTS = PB / PPW;
  constexpr int NT = SLOTS * LP;
  constexpr int MS = NT / PB;
  constexpr int CIT = (n + MS - 1) / MS;
  __shared__ Cx<T> lds[PB * BUF];
  const int tid = threadIdx.x;
  const int slot = tid / LP;
  const int lane = tid - slot * LP;
  const int tq = tid % PB;
  const int m0 = tid / PB;
  const int ldl = int(g.ld_line);
  const T scale = T(1.0 / sqrt(double(L)));
  typename Ln::Tw twl;
  twl.load(tw, lane);
  Cx<T>* ltile = lds + tq * BUF + m0;
  auto tile_ptr = [&](int t) -> Cx<T>* {
    const int tx = t % ntx;
    const int outer = t / ntx;
    return reinterpret_cast<Cx<T>*>(W + int64_t(outer) * g.ld_outer + tx * 2 * PB + m0 * ldl + 2 * tq);
  };
  Cx<T> pre[CIT];
  int t = first_tile<T, PB>();
  if (t < ntiles) {
    const Cx<T>* gp = tile_ptr(t);
#pragma unroll
    for (int it = 0; it < CIT; ++it)
      if (m0 + MS * it < n) pre[it] = gp[(MS * it * ldl) / 2];
  }
  for (; t < ntiles; t += gridDim.x) {
    const int cpair = (t % ntx) * 2 * PB + 2 * tq;  // first column of this thread's pair
#pragma unroll
    for (int it = 0; it < CIT; ++it)
      if (m0 + MS * it < n) ltile[MS * it] = mask_pad(pre[it], cpair, g.ncols);
    __syncthreads();
    const int tn = t + gridDim.x;
    if (tn < ntiles) {
      const Cx<T>* gp = tile_ptr(tn);
#pragma unroll
      for (int it = 0; it < CIT; ++it)
        if (m0 + MS * it < n) pre[it] = gp[(MS * it * ldl) / 2];
    }
    typename Ln::Regs v;
#pragma unroll 1
    for (int r = 0; r < PPW; ++r) {
      Cx<T>* my = lds + (slot + SLOTS * r) * BUF;
      Ln::transform(v, my, my, lane, twl, tw);
      Ln::outputs(v, lane, tw, [&](int k, Cx<T> Z) { my[k - 1] = Cx<T>{-Z.im * scale, Z.re * scale}; });
    }
    __syncthreads();
    Cx<T>* gd = tile_ptr(t);
#pragma unroll
    for (int it = 0; it < CIT; ++it)
      if (m0 + MS * it < n) gd[(MS * it * ldl) / 2] = mask_pad(ltile[MS * it], cpair, g.ncols);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Persistent, software-pipelined column pass with the diagonal stage (single
// grids with many column tiles).  Per tile: forward transform, stage, inverse
// transform, as in col_fast.  After the stage, the W values of the block's next
// tile are loaded into registers, so their latency hides behind the inverse
// transform and the tile's stores.  H is read inside the stage: holding the
// next tile's H values too exceeds the 128 registers per lane that 4 waves per
// SIMD leave (the FP64 stage spills), and measured slower.
template <typename T, int L, int PB, int PPW, int MODE, bool BAT = false>
__global__ void __launch_bounds__((PB / PPW * Line<T, L>::LP), (MinWaves<T, L>::value))
    col_stage_pipe(T* __restrict__ W, T* __restrict__ H, ColGeom g, const Cx<T>* tw, Diag dg, int ntx, int ntiles,
                   const ColInst<T>* __restrict__ insts, int tiles_per_inst) {
  using Ln = Line<T, L>;
  constexpr int N = L / 2;
  constexpr int n = N - 1;
  constexpr int LP = Ln::LP;
  constexpr int BUF = Ln::BUF;
  constexpr int SLOTS = PB / PPW;
  constexpr int NT = SLOTS * LP;
  constexpr int MS = NT / PB;
  constexpr int CIT = (n + MS - 1) / MS;
  __shared__ Cx<T> lds[PB * BUF];
  const int tid = threadIdx.x;
  const int slot = tid / LP;
  const int lane = tid - slot * LP;
  const int tq = tid % PB;
  const int m0 = tid / PB;
  const int ldl = int(g.ld_line);
  const T scale = T(1.0 / sqrt(double(L)));
  const double tau = dg.tau;
  const double rtc2 = 1.0 / (tau * dg.c2);
  typename Ln::Tw twl;
  twl.load(tw, lane);
  Cx<T>* ltile = lds + tq * BUF + m0;
  // tile t: instance t / tiles_per_inst of a batched launch (else the grid),
  // outer index and column tile of the rest
  auto inst_of = [&](int t) { return BAT ? t / tiles_per_inst : 0; };
  auto local = [&](int t) { return BAT ? t - inst_of(t) * tiles_per_inst : t; };
  auto wbase = [&](int t) -> T* { return BAT ? insts[inst_of(t)].W : W; };
  // element offset of this thread's first tile value (pair tq, row m0) in tile t
  auto offset = [&](int t) -> int64_t {
    const int lt = local(t);
    return int64_t(lt / ntx) * g.ld_outer + ((lt % ntx) * 2 * PB + m0 * ldl + 2 * tq);
  };
  Cx<T> pw[CIT];
  int t = first_tile<T, PB>();
  if (t < ntiles) {
    const Cx<T>* gw = reinterpret_cast<const Cx<T>*>(wbase(t) + offset(t));
#pragma unroll
    for (int it = 0; it < CIT; ++it)
      if (m0 + MS * it < n) pw[it] = gw[(MS * it * ldl) / 2];
  }
  for (; t < ntiles; t += gridDim.x) {
    const int lt = local(t);
    const int outer = lt / ntx;
    const int kx0 = (lt % ntx) * 2 * PB + 2 * tq;  // first column of this thread's pair
    const int64_t off = offset(t);
    T* const Wt = wbase(t);
    T* const Ht = BAT ? insts[inst_of(t)].H : H;
    // per-instance tables of a batched launch are held in separate locals
    AxisTab ta0 = dg.ax[0], ta1 = dg.ax[1], ta2 = dg.ax[2];
    double D = dg.D;
    if constexpr (BAT) {
      const ColInst<T>& I = insts[inst_of(t)];
      ta0 = I.ax[0];
      ta1 = I.ax[1];
      ta2 = I.ax[2];
      D = I.D;
    }
    const AxisTab line_tab = g.last_is_z ? ta2 : ta1;
#pragma unroll
    for (int it = 0; it < CIT; ++it)
      if (m0 + MS * it < n) ltile[MS * it] = mask_pad(pw[it], kx0, g.ncols);
    __syncthreads();
    const int tn = t + gridDim.x;
    typename Ln::Regs v;
#pragma unroll 1
    for (int r = 0; r < PPW; ++r) {
      Cx<T>* my = lds + (slot + SLOTS * r) * BUF;
      Ln::transform(v, my, my, lane, twl, tw);
      Ln::outputs(v, lane, tw, [&](int k, Cx<T> Z) { my[k - 1] = Cx<T>{-Z.im * scale, Z.re * scale}; });
    }
    __syncthreads();
    {
      // diagonal stage: thread -> (rows m0 + MS it, pair tq)
      Sep sxy[2];
      const Sep so = g.last_is_z ? sep_load(ta1, outer) : sep_load(ta2, 0);
      sxy[0] = sep_combine(sep_load(ta0, kx0), so);
      sxy[1] = sep_combine(sep_load(ta0, kx0 + 1), so);
      Cx<T>* hrow = reinterpret_cast<Cx<T>*>(Ht + off);
#pragma unroll
      for (int it = 0; it < CIT; ++it) {
        const int m = m0 + MS * it;
        if (m < n) {
          const Sep sl = sep_load(line_tab, m);
          const Cx<T> gv = ltile[MS * it];
          double o0, o1, n0, n1;
          const Cx<T> hh = hrow[(MS * it * ldl) / 2];
          diag_fast<MODE>(sep_combine(sxy[0], sl), D, tau, rtc2, double(gv.re), double(hh.re), &o0, &n0);
          diag_fast<MODE>(sep_combine(sxy[1], sl), D, tau, rtc2, double(gv.im), double(hh.im), &o1, &n1);
          hrow[(MS * it * ldl) / 2] = mask_pad(Cx<T>{T(n0), T(n1)}, kx0, g.ncols);
          ltile[MS * it] = Cx<T>{T(o0), T(o1)};
        }
      }
    }
    if (tn < ntiles) {
      const Cx<T>* gw = reinterpret_cast<const Cx<T>*>(wbase(tn) + offset(tn));
#pragma unroll
      for (int it = 0; it < CIT; ++it)
        if (m0 + MS * it < n) pw[it] = gw[(MS * it * ldl) / 2];
    }
    __syncthreads();
#pragma unroll 1
    for (int r = 0; r < PPW; ++r) {
      Cx<T>* my = lds + (slot + SLOTS * r) * BUF;
      Ln::transform(v, my, my, lane, twl, tw);
      Ln::outputs(v, lane, tw, [&](int k, Cx<T> Z) { my[k - 1] = Cx<T>{-Z.im * scale, Z.re * scale}; });
    }
    __syncthreads();
    Cx<T>* gd = reinterpret_cast<Cx<T>*>(Wt + off);
#pragma unroll
    for (int it = 0; it < CIT; ++it)
      if (m0 + MS * it < n) gd[(MS * it * ldl) / 2] = mask_pad(ltile[MS * it], kx0, g.ncols);
    __syncthreads();
  }
}


// ---------------------------------------------------------------------------
// Periodic lines of N = L points (L a power of two, 128 ... 1024): the real
// orthonormal Fourier transform of two packed lines through one complex FFT
// of length L, wave-local as above.  Forward: Z = FFT(a + ib), then position r
// of the half-complex order combines Z_r and Z_{L-r} (per_pos below); inverse:
// the FFT input at m is conj(Z^_m), built from the coefficients at m and L - m,
// and the nodal values are (X.re, -X.im) / sqrt(L).  Both pair reads go
// through the pair's LDS region.

// Coefficient pair at position m from the FFT outputs Z (line[k] = Z_k).
template <typename T, int L>
__device__ __forceinline__ Cx<T> per_pos(const Cx<T>* line, int m) {
  const T s1 = T(1.0 / sqrt(double(L)));
  const T s2 = T(1.0 / sqrt(2.0 * double(L)));
  if (m == 0 || 2 * m == L) {
    const Cx<T> z = line[m];
    return Cx<T>{z.re * s1, z.im * s1};
  }
  const Cx<T> zm = line[m], zo = line[L - m];
  if (2 * m < L) return Cx<T>{(zm.re + zo.re) * s2, (zm.im + zo.im) * s2};
  return Cx<T>{(zm.im - zo.im) * s2, (zo.re - zm.re) * s2};
}

// FFT input at m of the inverse transform: conj(Z^_m) from the coefficient
// pairs c at positions m and L - m.
template <typename T, int L>
__device__ __forceinline__ Cx<T> per_inv_input(const Cx<T>* c, int m) {
  const T r2 = T(0.70710678118654752440);
  if (m == 0 || 2 * m == L) {
    const Cx<T> v = c[m];
    return Cx<T>{v.re, -v.im};
  }
  if (2 * m < L) {
    const Cx<T> ck = c[m], cm = c[L - m];
    return Cx<T>{(ck.re + cm.im) * r2, (cm.re - ck.im) * r2};
  }
  const Cx<T> ck = c[L - m], cm = c[m];
  return Cx<T>{(ck.re - cm.im) * r2, -(ck.im + cm.re) * r2};
}

// Forward (INV = false: FFT of node[0 .. L-1]) or inverse (INV = true: FFT of
// the conj(Z^) built from the coefficient line node) transform of one pair;
// the region may overlay node (all inputs are read before it is written).
template <typename T, int L, bool INV>
__device__ __forceinline__ void per_fft(Cx<T> (&v)[FftShape<L>::E], const Cx<T>* node, Cx<T>* buf, int lane,
                                        const LaneTw<T, L>& tw) {
  constexpr int E = FftShape<L>::E;
  constexpr int LP = FftShape<L>::LP;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int m = lane + LP * q;
    v[q] = INV ? per_inv_input<T, L>(node, m) : node[m];
  }
  wave_sync();
  fft_head<T, L>(v, buf, lane);
  wave_sync();
  fft_tail<T, L>(v, buf, lane, tw);
  wave_sync();
}

// Visit every output k in [0, L) held by this lane: f(k, Z_k).
template <typename T, int L, typename F>
__device__ __forceinline__ void for_all_outputs(const Cx<T> (&v)[FftShape<L>::E], int lane, F f) {
  constexpr int E = FftShape<L>::E;
  constexpr int LP = FftShape<L>::LP;
  constexpr int R2 = FftShape<L>::R2;
  constexpr int NB = E / R2;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int q = 0; q < R2; ++q) f(lane + LP * b + q * (L / R2), v[b * R2 + q]);
  }
}

// Row pass of periodic x lines: ROW_FWD_USER, ROW_INV_USER or ROW_PHYS (as
// row_fast; the reaction takes no position, periodic grids have none).
template <typename T, int L, int PB, int MODE>
__global__ void __launch_bounds__((PB * FftShape<L>::LP), (MinWaves<T, L>::value)) row_fast_per(
    const T* src, T* dst, T* dst2, RowGeom g, const Cx<T>* __restrict__ tw, Forcing F) {
  constexpr int LP = FftShape<L>::LP;
  constexpr int BUF = FftShape<L>::BUF;
  constexpr int RIT = L / LP;
  __shared__ Cx<T> lds[PB * BUF];
  const int tid = threadIdx.x;
  const int p = tid / LP;
  const int lane = tid - p * LP;
  const int ra = blockIdx.x * 2 * PB + 2 * p, rb = ra + 1;
  const bool hasa = ra < g.nrows, hasb = rb < g.nrows;
  const T s1 = T(1.0 / sqrt(double(L)));
  LaneTw<T, L> twl;
  twl.load(tw, lane);
  Cx<T>* my = lds + p * BUF;
  {
    const T* sa = src + int64_t(ra) * g.ld_src + lane;
    const T* sb = src + int64_t(rb) * g.ld_src + lane;
    T va[RIT], vb[RIT];
#pragma unroll
    for (int t = 0; t < RIT; ++t) {
      va[t] = hasa ? sa[LP * t] : T(0);
      vb[t] = hasb ? sb[LP * t] : T(0);
    }
#pragma unroll
    for (int t = 0; t < RIT; ++t) my[lane + LP * t] = Cx<T>{va[t], vb[t]};
  }
  wave_sync();
  Cx<T> v[FftShape<L>::E];
  if (MODE != ROW_FWD_USER) {
    per_fft<T, L, true>(v, my, my, lane, twl);
    for_all_outputs<T, L>(v, lane, [&](int k, Cx<T> X) {
      const T ua = X.re * s1, ub = -X.im * s1;
      if (MODE == ROW_INV_USER)
        my[k] = Cx<T>{ua, ub};
      else
        my[k] = Cx<T>{reaction_k<T, RK_GENERIC>(F, ua, k, 0, 0), reaction_k<T, RK_GENERIC>(F, ub, k, 0, 0)};
    });
    wave_sync();
  }
  if (MODE != ROW_INV_USER) {
    per_fft<T, L, false>(v, my, my, lane, twl);
    for_all_outputs<T, L>(v, lane, [&](int k, Cx<T> Z) { my[k] = Z; });
    wave_sync();
  }
  Cx<T> outv[RIT];
#pragma unroll
  for (int t = 0; t < RIT; ++t) outv[t] = MODE == ROW_INV_USER ? my[lane + LP * t] : per_pos<T, L>(my, lane + LP * t);
  T* da = dst + int64_t(ra) * g.ld_dst + lane;
  T* db = dst + int64_t(rb) * g.ld_dst + lane;
#pragma unroll
  for (int t = 0; t < RIT; ++t) {
    if (hasa) da[LP * t] = outv[t].re;
    if (hasb) db[LP * t] = outv[t].im;
  }
  if (MODE == ROW_FWD_USER) {
    T* ha = dst2 + int64_t(ra) * g.ld_dst + lane;
    T* hb = dst2 + int64_t(rb) * g.ld_dst + lane;
#pragma unroll
    for (int t = 0; t < RIT; ++t) {
      if (hasa) ha[LP * t] = outv[t].re;
      if (hasb) hb[LP * t] = outv[t].im;
    }
  }
}

// Column pass of periodic lines (one tile of C = 2 PB columns per block, as
// col_fast): COL_PLAIN (forward), COL_PLAIN_INV (inverse) or a stage
// (forward, the diagonal stage at every position, inverse).
// The stage variants keep a tile column of results in registers between the
// two transforms: 2 waves per SIMD.
template <typename T, int L, int MODE>
struct PerMinWaves {
  static constexpr int value = (MODE == COL_PLAIN || MODE == COL_PLAIN_INV) ? MinWaves<T, L>::value : 2;
};

template <typename T, int L, int PB, int PPW, int MODE>
__global__ void __launch_bounds__((PB / PPW * FftShape<L>::LP), (PerMinWaves<T, L, MODE>::value)) col_fast_per(
    T* W, T* H, ColGeom g, const Cx<T>* tw, Diag dg) {
  constexpr int LP = FftShape<L>::LP;
  constexpr int BUF = FftShape<L>::BUF;
  constexpr int SLOTS = PB / PPW;
  constexpr int NT = SLOTS * LP;
  constexpr int MS = NT / PB;
  constexpr int CIT = (L + MS - 1) / MS;
  __shared__ Cx<T> lds[PB * BUF];
  const int tid = threadIdx.x;
  int bx, by, bz;
  tile_coords<T, PB>(bx, by, bz);
  const int c0 = bx * 2 * PB;
  const int outer = by;
  const int64_t base = int64_t(outer) * g.ld_outer + c0;
  const T s1 = T(1.0 / sqrt(double(L)));
  const int slot = tid / LP;
  const int lane = tid - slot * LP;
  const int tq = tid % PB;
  const int m0 = tid / PB;
  const int ldl = int(g.ld_line);
  Cx<T>* ltile = lds + tq * BUF;  // this thread's column pair, row m at ltile[m]
  {
    const Cx<T>* gsrc = reinterpret_cast<const Cx<T>*>(W + base + m0 * ldl + 2 * tq);
    Cx<T> tmp[CIT];
#pragma unroll
    for (int it = 0; it < CIT; ++it)
      if (m0 + MS * it < L) tmp[it] = gsrc[(MS * it * ldl) / 2];
#pragma unroll
    for (int it = 0; it < CIT; ++it)
      if (m0 + MS * it < L) ltile[m0 + MS * it] = mask_pad(tmp[it], c0 + 2 * tq, g.ncols);
  }
  __syncthreads();
  LaneTw<T, L> twl;
  twl.load(tw, lane);
  Cx<T> v[FftShape<L>::E];
  if (MODE == COL_PLAIN_INV) {
#pragma unroll 1
    for (int r = 0; r < PPW; ++r) {
      Cx<T>* my = lds + (slot + SLOTS * r) * BUF;
      per_fft<T, L, true>(v, my, my, lane, twl);
      for_all_outputs<T, L>(v, lane, [&](int k, Cx<T> X) { my[k] = Cx<T>{X.re * s1, -X.im * s1}; });
    }
  } else {
#pragma unroll 1
    for (int r = 0; r < PPW; ++r) {
      Cx<T>* my = lds + (slot + SLOTS * r) * BUF;
      per_fft<T, L, false>(v, my, my, lane, twl);
      for_all_outputs<T, L>(v, lane, [&](int k, Cx<T> Z) { my[k] = Z; });
    }
  }
  __syncthreads();
  if (MODE == COL_PLAIN || MODE == COL_PLAIN_INV) {
    Cx<T>* gdst = reinterpret_cast<Cx<T>*>(W + base + m0 * ldl + 2 * tq);
#pragma unroll
    for (int it = 0; it < CIT; ++it) {
      const int m = m0 + MS * it;
      if (m < L) {
        const Cx<T> c = MODE == COL_PLAIN ? per_pos<T, L>(ltile, m) : ltile[m];
        gdst[(MS * it * ldl) / 2] = mask_pad(c, c0 + 2 * tq, g.ncols);
      }
    }
    return;
  }
  // diagonal stage: thread -> (row m, pair tq); the coefficient pairs are read
  // from the FFT outputs before any is overwritten
  const double tau = dg.tau, c2 = dg.c2, D = dg.D;
  const int kx0 = c0 + 2 * tq;
  Sep sxy[2];
  {
    const Sep so = g.last_is_z ? sep_load(dg.ax[1], outer) : sep_load(dg.ax[2], 0);
    sxy[0] = sep_combine(sep_load(dg.ax[0], kx0), so);
    sxy[1] = sep_combine(sep_load(dg.ax[0], kx0 + 1), so);
  }
  const AxisTab line_tab = g.last_is_z ? dg.ax[2] : dg.ax[1];
  Cx<T>* hrow = reinterpret_cast<Cx<T>*>(H + base + m0 * ldl + 2 * tq);
  Cx<T> res[CIT];
#pragma unroll
  for (int it = 0; it < CIT; ++it) {
    const int m = m0 + MS * it;
    if (m < L) {
      const Cx<T> gv = per_pos<T, L>(ltile, m);
      const Cx<T> hv = hrow[(MS * it * ldl) / 2];
      const Sep sl = sep_load(line_tab, m);
      double o0, o1, n0, n1;
      if (MODE == COL_ETD1) {
        diag_apply<DIAG_ETD1>(sep_combine(sxy[0], sl), D, tau, c2, double(gv.re), double(hv.re), &o0, &n0);
        diag_apply<DIAG_ETD1>(sep_combine(sxy[1], sl), D, tau, c2, double(gv.im), double(hv.im), &o1, &n1);
      } else if (MODE == COL_STAGE_A) {
        diag_apply<DIAG_A>(sep_combine(sxy[0], sl), D, tau, c2, double(gv.re), double(hv.re), &o0, &n0);
        diag_apply<DIAG_A>(sep_combine(sxy[1], sl), D, tau, c2, double(gv.im), double(hv.im), &o1, &n1);
      } else {
        diag_apply<DIAG_B>(sep_combine(sxy[0], sl), D, tau, c2, double(gv.re), double(hv.re), &o0, &n0);
        diag_apply<DIAG_B>(sep_combine(sxy[1], sl), D, tau, c2, double(gv.im), double(hv.im), &o1, &n1);
      }
      hrow[(MS * it * ldl) / 2] = mask_pad(Cx<T>{T(n0), T(n1)}, kx0, g.ncols);
      res[it] = Cx<T>{T(o0), T(o1)};
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < CIT; ++it)
    if (m0 + MS * it < L) ltile[m0 + MS * it] = res[it];
  __syncthreads();
#pragma unroll 1
  for (int r = 0; r < PPW; ++r) {
    Cx<T>* my = lds + (slot + SLOTS * r) * BUF;
    per_fft<T, L, true>(v, my, my, lane, twl);
    for_all_outputs<T, L>(v, lane, [&](int k, Cx<T> X) { my[k] = Cx<T>{X.re * s1, -X.im * s1}; });
  }
  __syncthreads();
  Cx<T>* gdst = reinterpret_cast<Cx<T>*>(W + base + m0 * ldl + 2 * tq);
#pragma unroll
  for (int it = 0; it < CIT; ++it)
    if (m0 + MS * it < L) gdst[(MS * it * ldl) / 2] = mask_pad(ltile[m0 + MS * it], kx0, g.ncols);
}

}  // namespace fast
}  // namespace eife

// Sine-transform passes for long lines: N = 1024, 2048 and 4096 intervals
// (complex FFTs of L = 2048, 4096 and 8192 points of the odd extension of a
// line pair, as in Section 4's per-dimension transforms; the packing is the one
// of eife_kernels.hpp).
//
// A wavefront cannot hold such a line, so one block transforms one line pair:
// NT = L / 16 threads with 16 complex values each, Stockham stages of radix 16
// (16^3 = 4096; a 2048-point line ends with a radix-8 stage, an 8192-point line
// adds a final radix-2 stage) whose exchanges go through the pair's LDS buffer
// with block barriers, and the last stage's outputs left in registers.  The
// generic passes do every stage as a full LDS sweep; here the values stay in
// registers between exchanges.  Each thread loads its twiddle generators once
// per kernel (two per radix-16 stage, one for the last stage) and forms the
// powers for each stage by products at most three deep, so no stage waits on
// a table load.
#pragma once

#include "eife_kernels.hpp"
#include "eife_fast.hpp"

namespace eife {
namespace lng {

using fast::DftN;
using fast::xpad;

template <int L>
struct Shape {
  static constexpr int E = 16;                        // complex values per thread
  static constexpr int NT = L / E;                    // threads per line pair
  static constexpr int BUF = ((L + L / 8 + 63) / 64) * 64 + 2;  // padded exchange buffer
  static constexpr int RL = (L == 8192) ? 2 : (L == 2048 ? 8 : 16);  // radix of the last stage
  static_assert(L == 2048 || L == 4096 || L == 8192, "long-line passes: 2048, 4096 or 8192 FFT points");
};

// Registers per thread: FP32 8192-point lines fit 4 waves per SIMD (two blocks
// per compute unit); the other shapes take what they need (FP32 2048-point
// stage passes spill at 4).
template <typename T, int L>
struct LongWaves {
  static constexpr int value = (sizeof(T) == 4 && L == 8192) ? 4 : 1;
};

// Twiddle generators of one thread (tw[i] = exp(-2 pi i i / L)): for the
// stage after Ns = 16 points (radix 16) and the one after Ns = 256 (radix 16,
// or 8 when L = 2048), g = W_L^{k S} and g4 = W_L^{4 k S} with k = t mod Ns
// and S = L / (Ns R); for the radix-2 stage after Ns = 4096 (L = 8192), W_L^t.
template <typename T, int L>
struct LongTw {
  Cx<T> a1, a4, b1, b4, c1;
  __device__ __forceinline__ LongTw(const Cx<T>* __restrict__ tw, int t) {
    constexpr int SA = L / 256;
    constexpr int RB = L == 2048 ? 8 : 16;
    constexpr int SB = L / (256 * RB);
    a1 = tw[(t & 15) * SA];
    a4 = tw[4 * (t & 15) * SA];
    b1 = tw[(t & 255) * SB];
    b4 = tw[4 * (t & 255) * SB];
    c1 = L == 8192 ? tw[t] : Cx<T>{T(1), T(0)};
  }
};

// Makes the generators opaque to the optimiser, so that a second transform
// forms its powers again instead of keeping the first one's in registers.
template <typename T, int L>
__device__ __forceinline__ void refresh(LongTw<T, L>& gt) {
  asm volatile("" : "+v"(gt.a1.re), "+v"(gt.a1.im), "+v"(gt.a4.re), "+v"(gt.a4.im), "+v"(gt.b1.re), "+v"(gt.b1.im),
               "+v"(gt.b4.re), "+v"(gt.b4.im), "+v"(gt.c1.re), "+v"(gt.c1.im));
}

// p[q] = g^q, q = 1 .. R - 1 (R = 2, 8 or 16), from g and g4 = g^4: q = 4a + c
// as g4^a g^c.
template <typename T, int R>
__device__ __forceinline__ void gen_powers(Cx<T> g, Cx<T> g4, Cx<T> (&p)[R]) {
  p[1] = g;
  if constexpr (R > 2) {
    p[2] = cmul(g, g);
    p[3] = cmul(p[2], g);
    p[4] = g4;
  }
  if constexpr (R > 8) {
    p[8] = cmul(g4, g4);
    p[12] = cmul(p[8], g4);
  }
#pragma unroll
  for (int q = 5; q < R; ++q)
    if (q & 3) p[q] = cmul(p[q & ~3], p[q & 3]);
}

// Twiddle, butterflies and (unless LAST) the Stockham write of one stage of
// radix R after Ns points: butterfly j = t + NT b reads inputs j + (L/R) q,
// multiplies input q by W_{Ns R}^{(j mod Ns) q} = W_L^{(j mod Ns) q S}, S = L / (Ns R).
// The thread's powers p[q] = W_L^{(t mod Ns) q S} come from its generators g,
// g4; when NT < Ns, j mod Ns = t + NT b and the factor W_L^{NT b q S} is the
// same for every thread (a table load from a uniform address).
template <typename T, int L, int R, int Ns, bool LAST>
__device__ __forceinline__ void stage(Cx<T> (&v)[16], Cx<T>* buf, const Cx<T>* __restrict__ tw, Cx<T> g,
                                      Cx<T> g4, int t) {
  constexpr int NT = Shape<L>::NT;
  constexpr int NB = 16 / R;
  constexpr int S = L / (Ns * R);
  Cx<T> p[R];
  if constexpr (Ns > 1) gen_powers<T, R>(g, g4, p);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if constexpr (Ns > 1) {
      static_assert(NT % Ns == 0 || NT * NB <= Ns, "stage shape");
#pragma unroll
      for (int q = 1; q < R; ++q) {
        Cx<T> w = p[q];
        if constexpr (NT % Ns != 0)
          if (b > 0) w = cmul(w, tw[(NT * b * q * S) & (L - 1)]);
        v[b * R + q] = cmul(v[b * R + q], w);
      }
    }
    DftN<T, R>::run(&v[b * R]);
  }
  if constexpr (!LAST) {
    // output q of butterfly j goes to (j - k) R + k + Ns q (k = j mod Ns), padded
    // one slot every 8 (Ns is 1 or a multiple of 8, so every offset is exact)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = t + NT * b;
      const int k = j & (Ns - 1);
      Cx<T>* o = buf + xpad((j - k) * R + k);
#pragma unroll
      for (int q = 0; q < R; ++q) o[q * Ns + (q * Ns) / 8] = v[b * R + q];
    }
  }
}

// Inputs of a stage of radix R: v[b R + q] = buf at j + (L/R) q, j = t + NT b.
template <typename T, int L, int R>
__device__ __forceinline__ void gather(Cx<T> (&v)[16], const Cx<T>* buf, int t) {
  constexpr int NT = Shape<L>::NT;
  constexpr int S = L / R;
  const Cx<T>* rb = buf + xpad(t);
#pragma unroll
  for (int b = 0; b < 16 / R; ++b)
#pragma unroll
    for (int q = 0; q < R; ++q) v[b * R + q] = rb[(NT * b + S * q) + (NT * b + S * q) / 8];
}

// Forward FFT of length L of the odd extension of the pair whose values sit at
// node[0 .. N-2] (N = L / 2); node may overlay buf.  On return v[b RL + q] is
// output t + NT b + q (L / RL).  Every thread of the block takes part.
template <typename T, int L>
__device__ __forceinline__ void odd_fft(Cx<T> (&v)[16], const Cx<T>* node, Cx<T>* buf,
                                        const Cx<T>* __restrict__ tw, const LongTw<T, L>& gt, int t) {
  constexpr int NT = Shape<L>::NT;
  constexpr int N = L / 2;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int m = t + NT * q;  // m < N exactly for q < 8
    if (q < 8) {
      v[q] = (m == 0) ? Cx<T>{T(0), T(0)} : node[m - 1];
    } else if (m == N) {
      v[q] = Cx<T>{T(0), T(0)};
    } else {
      const Cx<T> c = node[2 * N - m - 1];
      v[q] = Cx<T>{-c.re, -c.im};
    }
  }
  __syncthreads();  // every node value is read before the buffer is written
  stage<T, L, 16, 1, false>(v, buf, tw, gt.a1, gt.a4, t);
  __syncthreads();
  gather<T, L, 16>(v, buf, t);
  __syncthreads();
  stage<T, L, 16, 16, false>(v, buf, tw, gt.a1, gt.a4, t);
  __syncthreads();
  if constexpr (L == 2048) {
    gather<T, L, 8>(v, buf, t);
    stage<T, L, 8, 256, true>(v, buf, tw, gt.b1, gt.b4, t);
    __syncthreads();  // the buffer may be rewritten next
    return;
  }
  gather<T, L, 16>(v, buf, t);
  if constexpr (L == 8192) {
    __syncthreads();
    stage<T, L, 16, 256, false>(v, buf, tw, gt.b1, gt.b4, t);
    __syncthreads();
    gather<T, L, 2>(v, buf, t);
    stage<T, L, 2, 4096, true>(v, buf, tw, gt.c1, gt.c1, t);
  } else {
    stage<T, L, 16, 256, true>(v, buf, tw, gt.b1, gt.b4, t);
  }
  __syncthreads();  // the buffer may be rewritten next
}

// The sine outputs k in [1, N-1] this thread holds: f(k, Z_k).
template <typename T, int L, typename F>
__device__ __forceinline__ void outputs(const Cx<T> (&v)[16], int t, F f) {
  constexpr int NT = Shape<L>::NT;
  constexpr int RL = Shape<L>::RL;
#pragma unroll
  for (int b = 0; b < 16 / RL; ++b)
#pragma unroll
    for (int q = 0; q < RL / 2; ++q) {
      const int k = t + NT * b + q * (L / RL);
      if (k >= 1) f(k, v[b * RL + q]);
    }
}

// The outputs k < N of a thread, numbered i = 0 .. COUNT-1: output index k(t, i)
// and its register slot (same set as outputs(), which also skips k = 0).
template <int L>
struct OutIdx {
  static constexpr int RL = Shape<L>::RL;
  static constexpr int COUNT = (16 / RL) * (RL / 2);
  static __device__ __forceinline__ int k(int t, int i) {
    return t + Shape<L>::NT * (i / (RL / 2)) + (i % (RL / 2)) * (L / RL);
  }
  static constexpr int slot(int i) { return (i / (RL / 2)) * RL + i % (RL / 2); }
};

// Row pass (x lines, contiguous): one line pair (rows 2 blockIdx.x, +1) per
// block; modes ROW_PHYS (inverse, reaction, forward), ROW_FWD_USER (forward of
// the caller's array into dst and dst2) and ROW_INV_USER (inverse into dst).
template <typename T, int L, int MODE, int RK>
__global__ void __launch_bounds__((Shape<L>::NT), (LongWaves<T, L>::value))
    row_long(const T* src, T* dst, T* dst2, RowGeom g, const Cx<T>* __restrict__ tw, Forcing F) {
  constexpr int NT = Shape<L>::NT;
  constexpr int N = L / 2;
  constexpr int n = N - 1;
  constexpr int RIT = (n + NT - 1) / NT;
  __shared__ Cx<T> lds[Shape<L>::BUF];
  const int t = threadIdx.x;
  const int ra = blockIdx.x * 2, rb = ra + 1;
  const bool hasb = rb < g.nrows;
  const T scale = T(1.0 / sqrt(double(L)));
  LongTw<T, L> gt(tw, t);
  {
    const T* sa = src + int64_t(ra) * g.ld_src + t;
    const T* sb = src + int64_t(rb) * g.ld_src + t;
    T va[RIT], vb[RIT];
#pragma unroll
    for (int i = 0; i < RIT; ++i) {
      const bool in = t + NT * i < n;
      va[i] = in ? sa[NT * i] : T(0);
      vb[i] = (in && hasb) ? sb[NT * i] : T(0);
    }
#pragma unroll
    for (int i = 0; i < RIT; ++i)
      if (t + NT * i < n) lds[t + NT * i] = Cx<T>{va[i], vb[i]};
  }
  __syncthreads();
  Cx<T> v[16];
  odd_fft<T, L>(v, lds, lds, tw, gt, t);
  if constexpr (MODE == ROW_PHYS) {
    const int iya = ra % g.ny, iza = ra / g.ny;
    const int iyb = rb % g.ny, izb = rb / g.ny;
    outputs<T, L>(v, t, [&](int k, Cx<T> Z) {
      const T ua = -Z.im * scale, ub = Z.re * scale;
      lds[k - 1] = Cx<T>{fast::reaction_k<T, RK>(F, ua, k - 1, iya, iza), fast::reaction_k<T, RK>(F, ub, k - 1, iyb, izb)};
    });
    __syncthreads();
    refresh(gt);
    odd_fft<T, L>(v, lds, lds, tw, gt, t);
  }
  outputs<T, L>(v, t, [&](int k, Cx<T> Z) { lds[k - 1] = Cx<T>{-Z.im * scale, Z.re * scale}; });
  __syncthreads();
  T* da = dst + int64_t(ra) * g.ld_dst + t;
  T* db = dst + int64_t(rb) * g.ld_dst + t;
  T* da2 = dst2 + int64_t(ra) * g.ld_dst + t;
  T* db2 = dst2 + int64_t(rb) * g.ld_dst + t;
#pragma unroll
  for (int i = 0; i < RIT; ++i) {
    if (t + NT * i < n) {
      const Cx<T> o = lds[t + NT * i];
      da[NT * i] = o.re;
      if (hasb) db[NT * i] = o.im;
      if constexpr (MODE == ROW_FWD_USER) {
        da2[NT * i] = o.re;
        if (hasb) db2[NT * i] = o.im;
      }
    }
  }
}

// Column pass (strided axis): one column pair (columns 2 bx, 2 bx + 1 at outer
// index by) per block, blocks in XCD-contiguous order so that the pairs of a
// 128-byte line share one L2.  COL_PLAIN: forward transform; COL_STAGE_A,
// COL_STAGE_B, COL_ETD1: forward, the diagonal stage with the spectral state H
// (its values for this thread's outputs loaded before the transform), inverse.
template <typename T, int L, int MODE>
__global__ void __launch_bounds__((Shape<L>::NT), (LongWaves<T, L>::value))
    col_long(T* W, T* H, ColGeom g, const Cx<T>* __restrict__ tw, Diag dg) {
  constexpr int NT = Shape<L>::NT;
  constexpr int N = L / 2;
  constexpr int n = N - 1;
  constexpr int RIT = (n + NT - 1) / NT;
  constexpr int NO = OutIdx<L>::COUNT;
  __shared__ Cx<T> lds[Shape<L>::BUF];
  const int t = threadIdx.x;
  int bx, outer;
  xcd_block(bx, outer);
  const int c0 = 2 * bx;
  const int64_t base = int64_t(outer) * g.ld_outer + c0;
  const T scale = T(1.0 / sqrt(double(L)));
  LongTw<T, L> gt(tw, t);
  Cx<T> hv[MODE == COL_PLAIN ? 1 : NO];
  if constexpr (MODE != COL_PLAIN) {
#pragma unroll
    for (int i = 0; i < NO; ++i) {
      const int k = OutIdx<L>::k(t, i);
      hv[i] = (k >= 1) ? *reinterpret_cast<const Cx<T>*>(H + base + int64_t(k - 1) * g.ld_line) : Cx<T>{T(0), T(0)};
    }
  }
#pragma unroll
  for (int i = 0; i < RIT; ++i) {
    const int m = t + NT * i;
    if (m < n)
      lds[m] = mask_pad(*reinterpret_cast<const Cx<T>*>(W + base + int64_t(m) * g.ld_line), c0, g.ncols);
  }
  __syncthreads();
  Cx<T> v[16];
  odd_fft<T, L>(v, lds, lds, tw, gt, t);
  if constexpr (MODE != COL_PLAIN) {
    const double tau = dg.tau, D = dg.D;
    const double rtc2 = 1.0 / (tau * dg.c2);
    const Sep sx0 = sep_load(dg.ax[0], c0), sx1 = sep_load(dg.ax[0], c0 + 1);
    const Sep so = g.last_is_z ? sep_load(dg.ax[1], outer) : sep_load(dg.ax[2], 0);
    const AxisTab line_tab = g.last_is_z ? dg.ax[2] : dg.ax[1];
    const Sep s0 = sep_combine(sx0, so), s1 = sep_combine(sx1, so);
#pragma unroll
    for (int i = 0; i < NO; ++i) {
      const int k = OutIdx<L>::k(t, i);
      if (k < 1) continue;
      const int m = k - 1;
      const Cx<T> Z = v[OutIdx<L>::slot(i)];
      const Sep sl = sep_load(line_tab, m);
      double o0, o1, n0, n1;
      fast::diag_fast<MODE>(sep_combine(s0, sl), D, tau, rtc2, double(-Z.im * scale), double(hv[i].re), &o0, &n0);
      fast::diag_fast<MODE>(sep_combine(s1, sl), D, tau, rtc2, double(Z.re * scale), double(hv[i].im), &o1, &n1);
      *reinterpret_cast<Cx<T>*>(H + base + int64_t(m) * g.ld_line) = mask_pad(Cx<T>{T(n0), T(n1)}, c0, g.ncols);
      lds[m] = Cx<T>{T(o0), T(o1)};
    }
    __syncthreads();
    refresh(gt);
    odd_fft<T, L>(v, lds, lds, tw, gt, t);
  }
  outputs<T, L>(v, t, [&](int k, Cx<T> Z) { lds[k - 1] = Cx<T>{-Z.im * scale, Z.re * scale}; });
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RIT; ++i) {
    const int m = t + NT * i;
    if (m < n) *reinterpret_cast<Cx<T>*>(W + base + int64_t(m) * g.ld_line) = mask_pad(lds[m], c0, g.ncols);
  }
}

// Columns c .. c + 3 of one row: one 16-byte access (FP32) or two adjacent
// 16-byte accesses (FP64).
template <typename T>
__device__ __forceinline__ void load4(const T* p, Cx<T>& a, Cx<T>& b) {
  if constexpr (sizeof(T) == 4) {
    const float4 w = *reinterpret_cast<const float4*>(p);
    a = Cx<T>{w.x, w.y};
    b = Cx<T>{w.z, w.w};
  } else {
    a = reinterpret_cast<const Cx<T>*>(p)[0];
    b = reinterpret_cast<const Cx<T>*>(p)[1];
  }
}
template <typename T>
__device__ __forceinline__ void store4(T* p, Cx<T> a, Cx<T> b) {
  if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<float4*>(p) = float4{a.re, a.im, b.re, b.im};
  } else {
    reinterpret_cast<Cx<T>*>(p)[0] = a;
    reinterpret_cast<Cx<T>*>(p)[1] = b;
  }
}

// Column pass over two adjacent column pairs per block: columns c0 .. c0+3 of
// a row are read and written as one piece (16 bytes FP32, 32 bytes FP64),
// which halves the memory requests of the strided axis against one pair per
// block.  Threads [0, NT) transform the first pair and [NT, 2 NT) the second,
// each in its own LDS buffer (two FP64 buffers fit up to 4096 points); the
// diagonal stage runs row by row over the sine coefficients both halves left
// in LDS, so H moves as whole row pieces as well.  Modes as col_long; blocks
// in XCD-contiguous order.
template <typename T, int L, int MODE>
__global__ void __launch_bounds__((2 * Shape<L>::NT), (LongWaves<T, L>::value))
    col_long4(T* W, T* H, ColGeom g, const Cx<T>* __restrict__ tw, Diag dg) {
  static_assert(2 * Shape<L>::BUF * sizeof(Cx<T>) <= 160 * 1024, "two pair buffers per block");
  constexpr int NT = Shape<L>::NT;
  constexpr int N = L / 2;
  constexpr int n = N - 1;
  constexpr int RIT = (n + 2 * NT - 1) / (2 * NT);
  __shared__ Cx<T> lds2[2][Shape<L>::BUF];
  const int half = int(threadIdx.x) / NT;  // uniform per wavefront (NT is a multiple of 64)
  const int t = int(threadIdx.x) - half * NT;
  const int tb = int(threadIdx.x);
  Cx<T>* lds = lds2[half];
  int bx, outer;
  xcd_block(bx, outer);
  const int c0 = 4 * bx;
  const int64_t base = int64_t(outer) * g.ld_outer + c0;
  const T scale = T(1.0 / sqrt(double(L)));
  LongTw<T, L> gt(tw, t);
#pragma unroll
  for (int i = 0; i < RIT; ++i) {
    const int m = tb + 2 * NT * i;
    if (m < n) {
      Cx<T> a, b;
      load4(W + base + int64_t(m) * g.ld_line, a, b);
      lds2[0][m] = mask_pad(a, c0, g.ncols);
      lds2[1][m] = mask_pad(b, c0 + 2, g.ncols);
    }
  }
  __syncthreads();
  Cx<T> v[16];
  odd_fft<T, L>(v, lds, lds, tw, gt, t);
  if constexpr (MODE != COL_PLAIN) {
    outputs<T, L>(v, t, [&](int k, Cx<T> Z) { lds[k - 1] = Cx<T>{-Z.im * scale, Z.re * scale}; });
    __syncthreads();
    const double tau = dg.tau, D = dg.D;
    const double rtc2 = 1.0 / (tau * dg.c2);
    const Sep so = g.last_is_z ? sep_load(dg.ax[1], outer) : sep_load(dg.ax[2], 0);
    const AxisTab line_tab = g.last_is_z ? dg.ax[2] : dg.ax[1];
#pragma unroll
    for (int i = 0; i < RIT; ++i) {
      const int m = tb + 2 * NT * i;
      if (m >= n) continue;
      Cx<T> ha, hb;
      load4(H + base + int64_t(m) * g.ld_line, ha, hb);
      const Cx<T> a = lds2[0][m], b = lds2[1][m];
      const Sep sl = sep_load(line_tab, m);
      const T gin[4] = {a.re, a.im, b.re, b.im};
      const T hin[4] = {ha.re, ha.im, hb.re, hb.im};
      T o[4], nh[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double oq, nq;
        fast::diag_fast<MODE>(sep_combine(sep_combine(sep_load(dg.ax[0], c0 + q), so), sl), D, tau, rtc2,
                              double(gin[q]), double(hin[q]), &oq, &nq);
        o[q] = T(oq);
        nh[q] = T(nq);
      }
      const Cx<T> h0 = mask_pad(Cx<T>{nh[0], nh[1]}, c0, g.ncols), h1 = mask_pad(Cx<T>{nh[2], nh[3]}, c0 + 2, g.ncols);
      store4(H + base + int64_t(m) * g.ld_line, h0, h1);
      lds2[0][m] = Cx<T>{o[0], o[1]};
      lds2[1][m] = Cx<T>{o[2], o[3]};
    }
    __syncthreads();
    refresh(gt);
    odd_fft<T, L>(v, lds, lds, tw, gt, t);
  }
  outputs<T, L>(v, t, [&](int k, Cx<T> Z) { lds[k - 1] = Cx<T>{-Z.im * scale, Z.re * scale}; });
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RIT; ++i) {
    const int m = tb + 2 * NT * i;
    if (m < n) {
      store4(W + base + int64_t(m) * g.ld_line, mask_pad(lds2[0][m], c0, g.ncols), mask_pad(lds2[1][m], c0 + 2, g.ncols));
    }
  }
}

}  // namespace lng
}  // namespace eife

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
  static constexpr int BUF = L + L / 8;           // padded exchange buffer (complex)
  static_assert(LP <= 64, "a line pair must fit in one wavefront");
  static_assert(R2 >= 2 && R2 <= E, "unsupported FFT length");
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One Stockham stage of radix R on the pair owned by this lane group.
// `in(i)` yields input i of the stage; unless LAST, the outputs are written
// to buf, else they stay in v (v[b*R+q] = output lane + LP*b + q*(L/R)).
template <typename T, int L, int R, int Ns, bool LAST, typename In>
__device__ __forceinline__ void wstage(Cx<T> (&v)[FftShape<L>::E], In in, Cx<T>* buf, int lane,
                                       const Cx<T>* __restrict__ tw) {
  constexpr int E = FftShape<L>::E;
  constexpr int LP = FftShape<L>::LP;
  constexpr int NB = E / R;
  constexpr int STRIDE = L / R;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lane + LP * b;
#pragma unroll
    for (int q = 0; q < R; ++q) v[b * R + q] = in(j + STRIDE * q, q);
    if (Ns > 1) {
      const int k = j & (Ns - 1);
#pragma unroll
      for (int q = 1; q < R; ++q) v[b * R + q] = cmul(v[b * R + q], tw[(q * k) * (L / (Ns * R))]);
    }
    DftN<T, R>::run(&v[b * R]);
  }
  if (!LAST) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = lane + LP * b;
      const int k = j & (Ns - 1);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) buf[xpad(base + q * Ns)] = v[b * R + q];
    }
  }
}

// Forward FFT of length L of the odd extension of the pair whose node values
// are given by get(i) (i = node index 0 .. N-2).  On return v holds the
// outputs (see wstage with LAST).
template <typename T, int L, typename Get>
__device__ __forceinline__ void odd_fft(Cx<T> (&v)[FftShape<L>::E], Get get, Cx<T>* buf, int lane,
                                        const Cx<T>* __restrict__ tw) {
  constexpr int E = FftShape<L>::E;
  constexpr int R2 = FftShape<L>::R2;
  constexpr int N = L / 2;
  auto in0 = [&](int m, int q) -> Cx<T> {
    // q < E/2  <=>  m < N  (m = j + (L/E) q with j < L/E)
    if (q < E / 2) {
      if (q == 0 && m == 0) return Cx<T>{T(0), T(0)};
      return get(m - 1);
    }
    if (q == E / 2 && m == N) return Cx<T>{T(0), T(0)};
    const Cx<T> c = get(2 * N - m - 1);
    return Cx<T>{-c.re, -c.im};
  };
  auto inb = [&](int i, int) -> Cx<T> { return buf[xpad(i)]; };
  wstage<T, L, E, 1, false>(v, in0, buf, lane, tw);
  wave_sync();
  wstage<T, L, E, E, false>(v, inb, buf, lane, tw);
  wave_sync();
  wstage<T, L, R2, E * E, true>(v, inb, buf, lane, tw);
  wave_sync();  // buf may be rewritten by the next transform of this pair
}

// Visit the outputs k in [1, N-1] held by this lane: f(k, Z_k).
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
// Row passes (x lines, contiguous).  Block = PB line pairs = 2 PB rows.
template <typename T, int L, int PB, int MODE>
__global__ void __launch_bounds__(PB * FftShape<L>::LP) row_fast(const T* src, T* dst, T* __restrict__ dst2,
                                                                  RowGeom g, const Cx<T>* __restrict__ tw, Forcing F) {
  constexpr int N = L / 2;
  constexpr int n = N - 1;
  constexpr int LP = FftShape<L>::LP;
  constexpr int E = FftShape<L>::E;
  constexpr int RS = N;  // tile row stride (complex)
  __shared__ Cx<T> tile[PB * RS];
  __shared__ Cx<T> xbuf[PB * FftShape<L>::BUF];
  const int tid = threadIdx.x;
  const int r0 = blockIdx.x * 2 * PB;
  const T scale = T(1.0 / sqrt(double(L)));

  // coalesced load of 2 PB rows into the pair-major tile
  for (int i = tid; i < 2 * PB * n; i += PB * LP) {
    const int row = i / n;
    const int m = i - row * n;
    const int r = r0 + row;
    const T val = (r < g.nrows) ? src[r * g.ld_src + m] : T(0);
    T* slot = reinterpret_cast<T*>(&tile[(row >> 1) * RS + m]);
    slot[row & 1] = val;
  }
  __syncthreads();

  const int p = tid / LP;
  const int lane = tid - p * LP;
  Cx<T>* my = tile + p * RS;
  Cx<T>* buf = xbuf + p * FftShape<L>::BUF;
  auto get = [&](int i) -> Cx<T> { return my[i]; };
  Cx<T> v[E];
  odd_fft<T, L>(v, get, buf, lane, tw);

  if (MODE == ROW_PHYS) {
    const int ra = r0 + 2 * p, rb = ra + 1;
    const int iya = ra % g.ny, iza = ra / g.ny;
    const int iyb = rb % g.ny, izb = rb / g.ny;
    for_outputs<T, L>(v, lane, [&](int k, Cx<T> Z) {
      const T ua = -Z.im * scale, ub = Z.re * scale;
      const T fa = reaction<T>(F, ua, k - 1, iya, iza);
      const T fb = (rb < g.nrows) ? reaction<T>(F, ub, k - 1, iyb, izb) : T(0);
      my[k - 1] = Cx<T>{fa, fb};
    });
    wave_sync();
    odd_fft<T, L>(v, get, buf, lane, tw);
  }
  for_outputs<T, L>(v, lane, [&](int k, Cx<T> Z) { my[k - 1] = Cx<T>{-Z.im * scale, Z.re * scale}; });
  __syncthreads();
  for (int i = tid; i < 2 * PB * n; i += PB * LP) {
    const int row = i / n;
    const int m = i - row * n;
    const int r = r0 + row;
    if (r < g.nrows) {
      const T val = reinterpret_cast<const T*>(&tile[(row >> 1) * RS + m])[row & 1];
      dst[r * g.ld_dst + m] = val;
      if (MODE == ROW_FWD_USER) dst2[r * g.ld_dst + m] = val;
    }
  }
}

// ---------------------------------------------------------------------------
// Column passes (strided axis).  Block = PB pairs = C = 2 PB adjacent x-columns.
template <typename T, int L, int PB, int MODE>
__global__ void __launch_bounds__(PB * FftShape<L>::LP) col_fast(T* __restrict__ W, T* __restrict__ H, ColGeom g,
                                                                  const Cx<T>* __restrict__ tw, Diag dg) {
  constexpr int N = L / 2;
  constexpr int n = N - 1;
  constexpr int LP = FftShape<L>::LP;
  constexpr int E = FftShape<L>::E;
  constexpr int NT = PB * LP;
  constexpr int TS = PB + 1;  // tile row stride (complex), padded against bank conflicts
  __shared__ Cx<T> tile[n * TS];
  __shared__ Cx<T> xbuf[PB * FftShape<L>::BUF];
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * 2 * PB;
  const int outer = blockIdx.y;
  const int64_t base = int64_t(outer) * g.ld_outer + c0;
  const T scale = T(1.0 / sqrt(double(L)));

  for (int i = tid; i < n * PB; i += NT) {
    const int m = i / PB;
    const int q = i - m * PB;
    tile[m * TS + q] = *reinterpret_cast<const Cx<T>*>(W + base + m * g.ld_line + 2 * q);
  }
  __syncthreads();

  const int p = tid / LP;
  const int lane = tid - p * LP;
  Cx<T>* buf = xbuf + p * FftShape<L>::BUF;
  auto get = [&](int i) -> Cx<T> { return tile[i * TS + p]; };
  Cx<T> v[E];
  odd_fft<T, L>(v, get, buf, lane, tw);
  for_outputs<T, L>(v, lane, [&](int k, Cx<T> Z) { tile[(k - 1) * TS + p] = Cx<T>{-Z.im * scale, Z.re * scale}; });

  if (MODE != COL_PLAIN) {
    __syncthreads();
    // diagonal stage over the tile: thread -> (row m, pair q), pair fixed per thread
    const double tau = dg.tau, c2 = dg.c2, D = dg.D;
    const int q = tid % PB;
    const int kx0 = c0 + 2 * q;
    Sep sxy[2];
    if (g.last_is_z) {
      const Sep sy = sep_load(dg.ax[1], outer);
      sxy[0] = sep_combine(sep_load(dg.ax[0], kx0), sy);
      sxy[1] = sep_combine(sep_load(dg.ax[0], kx0 + 1), sy);
    } else {
      const Sep sz = sep_load(dg.ax[2], 0);
      sxy[0] = sep_combine(sep_load(dg.ax[0], kx0), sz);
      sxy[1] = sep_combine(sep_load(dg.ax[0], kx0 + 1), sz);
    }
    const AxisTab& line_tab = g.last_is_z ? dg.ax[2] : dg.ax[1];
    for (int m = tid / PB; m < n; m += NT / PB) {
      const Sep sl = sep_load(line_tab, m);
      const Cx<T> gv = tile[m * TS + q];
      Cx<T>* hp = reinterpret_cast<Cx<T>*>(H + base + m * g.ld_line + 2 * q);
      const Cx<T> hv = *hp;
      double o0, o1, n0, n1;
      const Sep s0 = sep_combine(sxy[0], sl);
      const Sep s1 = sep_combine(sxy[1], sl);
      if (MODE == COL_ETD1) {
        diag_apply<DIAG_ETD1>(s0, D, tau, c2, double(gv.re), double(hv.re), &o0, &n0);
        diag_apply<DIAG_ETD1>(s1, D, tau, c2, double(gv.im), double(hv.im), &o1, &n1);
      } else if (MODE == COL_STAGE_A) {
        diag_apply<DIAG_A>(s0, D, tau, c2, double(gv.re), double(hv.re), &o0, &n0);
        diag_apply<DIAG_A>(s1, D, tau, c2, double(gv.im), double(hv.im), &o1, &n1);
      } else {
        diag_apply<DIAG_B>(s0, D, tau, c2, double(gv.re), double(hv.re), &o0, &n0);
        diag_apply<DIAG_B>(s1, D, tau, c2, double(gv.im), double(hv.im), &o1, &n1);
      }
      *hp = Cx<T>{T(n0), T(n1)};
      tile[m * TS + q] = Cx<T>{T(o0), T(o1)};
    }
    __syncthreads();
    odd_fft<T, L>(v, get, buf, lane, tw);
    for_outputs<T, L>(v, lane,
                      [&](int k, Cx<T> Z) { tile[(k - 1) * TS + p] = Cx<T>{-Z.im * scale, Z.re * scale}; });
  }
  __syncthreads();
  for (int i = tid; i < n * PB; i += NT) {
    const int m = i / PB;
    const int q = i - m * PB;
    *reinterpret_cast<Cx<T>*>(W + base + m * g.ld_line + 2 * q) = tile[m * TS + q];
  }
}

}  // namespace fast
}  // namespace eife

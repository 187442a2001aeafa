// Sine transforms as dense products on the matrix cores (split BF16).
//
// Along one axis the orthonormal sine transform is Y = S X with
// S_mk = sqrt(2/N) sin((m+1)(k+1) pi / N) (Section 4; the sqrt(2/N) scaling
// makes S symmetric and orthogonal, so one matrix serves both directions).
// Each FP32 operand is split into two BF16 parts, x = x_hi + x_lo with
// x_hi = bf16(x) and x_lo = bf16(x - x_hi), and S X is accumulated in FP32
// from the three products S_hi X_hi + S_hi X_lo + S_lo X_hi on
// v_mfma_f32_16x16x32_bf16; the dropped S_lo X_lo term and the rounding of the
// low parts leave a relative error of order 2^-16 per product.
//
// The pass structure is that of the FFT passes: a block owns TL complete lines
// (x rows for the row pass, adjacent x columns of one outer index for the
// column passes), so the reaction or the diagonal stage sits between the two
// products of a pass.  Lines are held in LDS as [line][k] BF16 hi/lo (the B
// operand); S is read from global memory as the A operand ([m][k] hi/lo, zero
// padded to KP x KP, small enough to stay in L2).  A wave owns MPW mode tiles
// and every line tile, so each S fragment it loads feeds LT products.
//
// MFMA 16x16x32 lane layout (checked on gfx950): lane l supplies A row l%16
// and B column l%16 with k = 8 (l/16) .. 8 (l/16) + 7, and receives
// D[4 (l/16) + r][l%16], r = 0..3.
#pragma once

#include <hip/hip_runtime.h>

#include "eife_kernels.hpp"
#include "eife_fast.hpp"

namespace eife {
namespace gemm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct SMat {
  const __bf16* hi;  // [KP][KP] row-major (m, k)
  const __bf16* lo;
};

// Lines per block for a padded length KP.
constexpr int lines_for(int KP) { return KP <= 256 ? 64 : 32; }

template <int KP>
struct Shape {
  static constexpr int TL = lines_for(KP);
  static constexpr int MT = KP / 16;                 // mode tiles
  static constexpr int WV = MT < 8 ? MT : 8;         // waves per block
  static constexpr int THREADS = WV * 64;
  static constexpr int MPW = MT / WV;                // mode tiles per wave
  static constexpr int LT = TL / 16;                 // line tiles (all owned by every wave)
  static constexpr int LS = KP + 8;                  // LDS line stride (bf16): 16-byte slots spread over banks
  static constexpr int OS = KP + 4;                  // FP32 staging stride, [line][mode] (row passes)
  static constexpr int TS = TL + 4;                  // FP32 staging stride, [mode][line] (column passes)
  static constexpr size_t LDS_B = size_t(2) * TL * LS * sizeof(__bf16);
  static constexpr size_t LDS_O = size_t(TL) * OS * sizeof(float);
  static constexpr size_t LDS_T = size_t(KP) * TS * sizeof(float);
  static constexpr size_t LDS_R = LDS_B > LDS_O ? LDS_B : LDS_O;
  static constexpr size_t LDS = LDS_R > LDS_T ? LDS_R : LDS_T;
  static_assert(KP % 32 == 0 && MT % WV == 0, "padded length");
};

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = __bf16(x);
  lo = __bf16(x - float(hi));
}

template <int KP>
struct Acc {
  f32x4 v[Shape<KP>::MPW][Shape<KP>::LT];
};

// acc = S * B over the block's lines for the wave's mode tiles.  PF: the S
// fragments of the next k step are loaded (from L2) while this step's products
// run (the passes whose stage code already needs more than 128 registers keep
// PF off: the extra registers would cost them a wave per SIMD, measured slower).
template <int KP, bool PF = true>
__device__ __forceinline__ void gemm_block(Acc<KP>& acc, const __bf16* bhi, const __bf16* blo, SMat S, int wave,
                                           int lane) {
  using Sh = Shape<KP>;
  const int kq = 8 * (lane >> 4);
  const int row = lane & 15;
#pragma unroll
  for (int i = 0; i < Sh::MPW; ++i)
#pragma unroll
    for (int t = 0; t < Sh::LT; ++t) acc.v[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  if constexpr (!PF) {
    for (int kk = 0; kk < KP; kk += 32) {
      bf16x8 xh[Sh::LT], xl[Sh::LT];
#pragma unroll
      for (int t = 0; t < Sh::LT; ++t) {
        const int o = (t * 16 + row) * Sh::LS + kk + kq;
        xh[t] = *reinterpret_cast<const bf16x8*>(bhi + o);
        xl[t] = *reinterpret_cast<const bf16x8*>(blo + o);
      }
#pragma unroll
      for (int i = 0; i < Sh::MPW; ++i) {
        const size_t off = size_t((wave + Sh::WV * i) * 16 + row) * KP + kk + kq;
        const bf16x8 sh = *reinterpret_cast<const bf16x8*>(S.hi + off);
        const bf16x8 sl = *reinterpret_cast<const bf16x8*>(S.lo + off);
#pragma unroll
        for (int t = 0; t < Sh::LT; ++t) {
          acc.v[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sh, xh[t], acc.v[i][t], 0, 0, 0);
          acc.v[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sh, xl[t], acc.v[i][t], 0, 0, 0);
          acc.v[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sl, xh[t], acc.v[i][t], 0, 0, 0);
        }
      }
    }
    return;
  }
  bf16x8 sh[Sh::MPW], sl[Sh::MPW];
  auto load_s = [&](int kk, bf16x8 (&h)[Sh::MPW], bf16x8 (&l)[Sh::MPW]) {
#pragma unroll
    for (int i = 0; i < Sh::MPW; ++i) {
      const size_t off = size_t((wave + Sh::WV * i) * 16 + row) * KP + kk + kq;
      h[i] = *reinterpret_cast<const bf16x8*>(S.hi + off);
      l[i] = *reinterpret_cast<const bf16x8*>(S.lo + off);
    }
  };
  load_s(0, sh, sl);
  for (int kk = 0; kk < KP; kk += 32) {
    bf16x8 shn[Sh::MPW], sln[Sh::MPW];
    if (kk + 32 < KP) load_s(kk + 32, shn, sln);
    bf16x8 xh[Sh::LT], xl[Sh::LT];
#pragma unroll
    for (int t = 0; t < Sh::LT; ++t) {
      const int o = (t * 16 + row) * Sh::LS + kk + kq;
      xh[t] = *reinterpret_cast<const bf16x8*>(bhi + o);
      xl[t] = *reinterpret_cast<const bf16x8*>(blo + o);
    }
#pragma unroll
    for (int i = 0; i < Sh::MPW; ++i) {
#pragma unroll
      for (int t = 0; t < Sh::LT; ++t) {
        acc.v[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sh[i], xh[t], acc.v[i][t], 0, 0, 0);
        acc.v[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sh[i], xl[t], acc.v[i][t], 0, 0, 0);
        acc.v[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sl[i], xh[t], acc.v[i][t], 0, 0, 0);
      }
    }
    if (kk + 32 < KP) {
#pragma unroll
      for (int i = 0; i < Sh::MPW; ++i) {
        sh[i] = shn[i];
        sl[i] = sln[i];
      }
    }
  }
}

// Visit the accumulator entries: f(mode m, line l, value&).
template <int KP, typename F>
__device__ __forceinline__ void for_acc(Acc<KP>& acc, int wave, int lane, F f) {
  using Sh = Shape<KP>;
#pragma unroll
  for (int i = 0; i < Sh::MPW; ++i)
#pragma unroll
    for (int t = 0; t < Sh::LT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float x = acc.v[i][t][r];
        f((wave + Sh::WV * i) * 16 + 4 * (lane >> 4) + r, t * 16 + (lane & 15), x);
        acc.v[i][t][r] = x;
      }
}

// Accumulators (modes >= n zeroed) -> BF16 hi/lo B operand of the next product.
template <int KP>
__device__ __forceinline__ void acc_to_b(const Acc<KP>& acc, __bf16* bhi, __bf16* blo, int n, int wave, int lane) {
  using Sh = Shape<KP>;
#pragma unroll
  for (int i = 0; i < Sh::MPW; ++i)
#pragma unroll
    for (int t = 0; t < Sh::LT; ++t) {
      const int m0 = (wave + Sh::WV * i) * 16 + 4 * (lane >> 4);
      const int o = (t * 16 + (lane & 15)) * Sh::LS + m0;
      bf16x4 h, l;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        __bf16 a, b;
        split_bf16(m0 + r < n ? acc.v[i][t][r] : 0.f, a, b);
        h[r] = a;
        l[r] = b;
      }
      *reinterpret_cast<bf16x4*>(bhi + o) = h;
      *reinterpret_cast<bf16x4*>(blo + o) = l;
    }
}

// Accumulators -> FP32 staging [line][mode].
template <int KP>
__device__ __forceinline__ void acc_to_stage(const Acc<KP>& acc, float* stage, int wave, int lane) {
  using Sh = Shape<KP>;
#pragma unroll
  for (int i = 0; i < Sh::MPW; ++i)
#pragma unroll
    for (int t = 0; t < Sh::LT; ++t) {
      const int m0 = (wave + Sh::WV * i) * 16 + 4 * (lane >> 4);
      *reinterpret_cast<f32x4*>(stage + (t * 16 + (lane & 15)) * Sh::OS + m0) = acc.v[i][t];
    }
}

// Accumulators -> FP32 staging [mode][line] (lanes of a row write adjacent lines).
template <int KP>
__device__ __forceinline__ void acc_to_stage_t(const Acc<KP>& acc, float* stage, int wave, int lane) {
  using Sh = Shape<KP>;
#pragma unroll
  for (int i = 0; i < Sh::MPW; ++i)
#pragma unroll
    for (int t = 0; t < Sh::LT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        stage[((wave + Sh::WV * i) * 16 + 4 * (lane >> 4) + r) * Sh::TS + t * 16 + (lane & 15)] = acc.v[i][t][r];
}

// ---------------------------------------------------------------------------
// Row passes over TL x-rows per block (modes as the FFT row passes):
//   ROW_PHYS      W -> S (f(S W)) in place (x-spectral in and out)
//   ROW_FWD_USER  dst = dst2 = S src
//   ROW_INV_USER  dst = S src
template <int KP, int MODE, bool AC>
__global__ void __launch_bounds__(Shape<KP>::THREADS) gemm_row(const float* src, float* dst, float* dst2, RowGeom g,
                                                               SMat S, Forcing F) {
  using Sh = Shape<KP>;
  constexpr int TL = Sh::TL;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  __bf16* bhi = reinterpret_cast<__bf16*>(smem_raw);
  __bf16* blo = bhi + TL * Sh::LS;
  float* stage = reinterpret_cast<float*>(smem_raw);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int n = g.n;
  const int r0 = blockIdx.x * TL;
  for (int i = tid; i < TL * KP; i += Sh::THREADS) {
    const int l = i / KP, k = i - l * KP;
    const int r = r0 + l;
    const float x = (k < n && r < g.nrows) ? src[int64_t(r) * g.ld_src + k] : 0.f;
    split_bf16(x, bhi[l * Sh::LS + k], blo[l * Sh::LS + k]);
  }
  __syncthreads();
  constexpr bool PF = AC || MODE != ROW_PHYS;
  Acc<KP> acc;
  gemm_block<KP, PF>(acc, bhi, blo, S, wave, lane);
  if (MODE == ROW_PHYS) {
    for_acc<KP>(acc, wave, lane, [&](int m, int l, float& v) {
      const int r = r0 + l;
      if (m < n && r < g.nrows) v = AC ? v - v * v * v : reaction<float, false>(F, v, m, r % g.ny, r / g.ny);
    });
    __syncthreads();
    acc_to_b<KP>(acc, bhi, blo, n, wave, lane);
    __syncthreads();
    gemm_block<KP, PF>(acc, bhi, blo, S, wave, lane);
  }
  __syncthreads();
  acc_to_stage<KP>(acc, stage, wave, lane);
  __syncthreads();
  for (int i = tid; i < TL * KP; i += Sh::THREADS) {
    const int l = i / KP, k = i - l * KP;
    const int r = r0 + l;
    if (k < n && r < g.nrows) {
      const float v = stage[l * Sh::OS + k];
      dst[int64_t(r) * g.ld_dst + k] = v;
      if (MODE == ROW_FWD_USER) dst2[int64_t(r) * g.ld_dst + k] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Column passes over TL adjacent x-columns of one outer index per block; line
// l is column c0 + l, its element k sits at base + k * ld_line + l.  Columns
// ncols .. pitch-1 are row padding and are written as exact zeros; columns
// from pitch on (the last block's overhang) are not touched.
template <int KP, int MODE>
__global__ void __launch_bounds__(Shape<KP>::THREADS) gemm_col(float* W, float* H, ColGeom g, int pitch, SMat S,
                                                               Diag dg) {
  using Sh = Shape<KP>;
  constexpr int TL = Sh::TL;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  __bf16* bhi = reinterpret_cast<__bf16*>(smem_raw);
  __bf16* blo = bhi + TL * Sh::LS;
  float* stage = reinterpret_cast<float*>(smem_raw);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int n = g.n;
  const int c0 = blockIdx.x * TL;
  const int outer = blockIdx.y;
  const int64_t base = int64_t(outer) * g.ld_outer + c0;
  // each thread gathers 8 consecutive k of one line (every load coalesced
  // across the lines) and writes them as one 16-byte hi and one lo vector
#pragma unroll
  for (int i = tid; i < TL * (KP / 8); i += Sh::THREADS) {
    const int l = i % TL, k0 = 8 * (i / TL);
    const bool ok = c0 + l < g.ncols;
    float x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = (ok && k0 + j < n) ? W[base + int64_t(k0 + j) * g.ld_line + l] : 0.f;
    bf16x8 h, lo;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      __bf16 a, b;
      split_bf16(x[j], a, b);
      h[j] = a;
      lo[j] = b;
    }
    *reinterpret_cast<bf16x8*>(bhi + l * Sh::LS + k0) = h;
    *reinterpret_cast<bf16x8*>(blo + l * Sh::LS + k0) = lo;
  }
  __syncthreads();
  constexpr bool PF = MODE == COL_PLAIN;
  Acc<KP> acc;
  gemm_block<KP, PF>(acc, bhi, blo, S, wave, lane);
  if (MODE != COL_PLAIN) {
    // diagonal stage: the x (and fixed outer-axis) factors of a lane's LT
    // columns are combined once, the line-axis factor per mode
    const double tau = dg.tau, D = dg.D, rtc2 = 1.0 / (tau * dg.c2);
    const Sep so = g.last_is_z ? sep_load(dg.ax[1], outer) : sep_load(dg.ax[2], 0);
    const AxisTab line_tab = g.last_is_z ? dg.ax[2] : dg.ax[1];  // a copy: no private-memory struct
    Sep sx[Sh::LT];
#pragma unroll
    for (int t = 0; t < Sh::LT; ++t) {
      const int kx = c0 + t * 16 + (lane & 15);
      sx[t] = sep_combine(sep_load(dg.ax[0], kx < g.ncols ? kx : 0), so);
    }
#pragma unroll
    for (int i = 0; i < Sh::MPW; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = (wave + Sh::WV * i) * 16 + 4 * (lane >> 4) + r;
        if (m >= n) continue;
        const Sep sl = sep_load(line_tab, m);
#pragma unroll
        for (int t = 0; t < Sh::LT; ++t) {
          const int l = t * 16 + (lane & 15);
          if (c0 + l >= g.ncols) continue;
          float* hp = H + base + int64_t(m) * g.ld_line + l;
          double o, nh;
          fast::diag_fast<MODE>(sep_combine(sx[t], sl), D, tau, rtc2, double(acc.v[i][t][r]), double(*hp), &o, &nh);
          *hp = float(nh);
          acc.v[i][t][r] = float(o);
        }
      }
    __syncthreads();
    acc_to_b<KP>(acc, bhi, blo, n, wave, lane);
    __syncthreads();
    gemm_block<KP, PF>(acc, bhi, blo, S, wave, lane);
  }
  __syncthreads();
  acc_to_stage_t<KP>(acc, stage, wave, lane);
  __syncthreads();
  for (int i = tid; i < TL * KP; i += Sh::THREADS) {
    const int k = i / TL, l = i - k * TL;
    if (k < n && c0 + l < pitch) W[base + int64_t(k) * g.ld_line + l] = (c0 + l < g.ncols) ? stage[k * Sh::TS + l] : 0.f;
  }
}

}  // namespace gemm
}  // namespace eife

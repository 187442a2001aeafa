// Host side of the EIFE library: the C ABI declared in include/eife.h.
//
// Per step the library runs the transform-scale-reaction-transform loop of
// Section 4 (eqs. (4.3)-(4.4)) on two device arrays owned by the grid:
//   W  the work array, spectral along x only between passes;
//   H  the spectral state u^ = S u (S the orthonormal sine transform along
//      every axis); during an EIFE2 step H holds E u^ + tau (phi_1 - phi_2/c2) G^_1.
// Passes (x fastest; the last axis is y in 2D and z in 3D):
//   row pass   inverse sine transform along x -> f(t, x, u) -> forward along x
//   mid pass   sine transform along y (3D only)
//   last pass  forward along the last axis -> diagonal phi stage -> inverse
// EIFE1 (eq. (2.13)): row, [mid], last(ETD1), [mid]             per step
// EIFE2 (eq. (2.14)): row, [mid], last(A), [mid], row, [mid], last(B), [mid]
// A 1D grid runs as a 2D grid with one virtual node along y whose tables make
// it the identity.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/eife.h"
#include "eife_kernels.hpp"
#include "eife_fast.hpp"

using namespace eife;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess) return fail(EIFE_EHIP, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

constexpr int kThreads = 256;
constexpr size_t kLdsBudget = 80 * 1024;  // per block, two blocks per CU fit in 160 KB
constexpr int kNormBlocksMax = 1024;
constexpr int kTabArrays = 5;  // lam, w, M, Q, Mc per axis
constexpr int kPipeBlocksPerCu = 4;  // resident blocks of the pipelined column pass (LDS permitting)
int g_cus = 256;                     // compute units of the device (set at grid creation)

bool factor_plan(int L, FftPlan* pl) {
  pl->L = L;
  pl->n4 = pl->n2 = pl->n3 = 0;
  int r = L;
  while (r % 4 == 0) {
    r /= 4;
    pl->n4++;
  }
  while (r % 2 == 0) {
    r /= 2;
    pl->n2++;
  }
  while (r % 3 == 0) {
    r /= 3;
    pl->n3++;
  }
  return r == 1;
}

}  // namespace

struct eife_grid_s {
  int d = 0;
  int N[3] = {2, 2, 2};
  int n[3] = {1, 1, 1};  // interior nodes per axis (virtual axes: 1)
  double h[3] = {1, 1, 1};
  double a[3] = {0, 0, 0};
  double D = 1;
  int dtype = EIFE_F64;
  size_t esz = 8;
  int pitch = 0;  // row pitch of W and H (elements)
  // scheme
  double tau = 0;
  int stages = 0;
  double c2 = 0.5;
  int load = EIFE_LOAD_LUMPED;
  double c0 = 0, c1 = 0;
  bool phi_ready = false;
  int device = 0;
  size_t max_lds = 65536;
  // device memory
  void* W = nullptr;
  void* H = nullptr;
  void* tw[3] = {nullptr, nullptr, nullptr};
  double* tab[3] = {nullptr, nullptr, nullptr};  // kTabArrays arrays per axis
  int tablen[3] = {0, 0, 0};
  double* partials = nullptr;
  double* out5 = nullptr;
  double* host5 = nullptr;  // pinned
  // launch shapes
  FftPlan plan[3];
  int transform = EIFE_TX_FFT;
  int prow = 1;     // pairs per block, row pass
  int pcol[3] = {1, 1, 1};  // pairs per block, column pass along axis 1, 2
  int nlines_total() const { return n[1] * n[2]; }
  // per-pass timing (eife_profile)
  bool prof_on = false;
  struct ProfRec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  double prof_ms[EIFE_PASS_COUNT] = {0};
  int64_t prof_n[EIFE_PASS_COUNT] = {0};
};

namespace {

size_t lds_bytes(const eife_grid_s* g, int P, int L) { return size_t(P) * size_t(L + 1) * 2 * g->esz; }

int pick_pairs(const eife_grid_s* g, int L, int cap) {
  int P = cap;
  while (P > 1 && (lds_bytes(g, P, L) > kLdsBudget || size_t(P) * L > size_t(kMaxElems) * kThreads)) P--;
  return P;
}

template <typename T>
void fill_twiddles(std::vector<Cx<T>>& v, int L) {
  v.resize(L);
  for (int j = 0; j < L; ++j) {
    const double ang = -2.0 * M_PI * double(j) / double(L);
    v[j] = Cx<T>{T(std::cos(ang)), T(std::sin(ang))};
  }
}

// lambda_k = lamB_k / lamA_k = 6 (1 - cos t) / (h^2 (2 + cos t)), t = k pi / N
// (Section 4, with the mass eigenvalue (h/6)(4 + 2 cos t)); 1 - cos t is
// formed as 2 sin^2(t/2) to avoid cancellation for small k.
double lam1d(int N, double h, int k) {
  const double t = double(k) * M_PI / double(N);
  const double s = std::sin(0.5 * t);
  return 12.0 * s * s / (h * h * (2.0 + std::cos(t)));
}

double lamA1d(int N, double h, int k) {
  const double t = double(k) * M_PI / double(N);
  return (h / 6.0) * (4.0 + 2.0 * std::cos(t));
}

// expm1(z) and expm1(z) - z for z <= 0 without cancellation: power series
// below |z| = 1/2, library expm1 above.
double expm1_minus_z(double z) {
  if (std::fabs(z) < 0.5) {
    double term = z * z / 2.0, sum = 0.0;
    for (int m = 2; m < 40 && term != 0.0; ++m) {
      sum += term;
      term *= z / double(m + 1);
    }
    return sum;
  }
  return std::expm1(z) - z;
}

int upload_tables(eife_grid_s* g) {
  for (int ax = 0; ax < 3; ++ax) {
    const int len = g->tablen[ax];
    std::vector<double> buf(kTabArrays * size_t(len), 0.0);
    double* lam = buf.data();
    double* w = lam + len;
    double* M = w + len;
    double* Q = M + len;
    double* Mc = Q + len;
    const bool real_axis = ax < g->d;
    for (int k = 0; k < len; ++k) {
      if (!real_axis) {  // virtual axis of a 1D/2D grid: the identity
        lam[k] = 0.0;
        w[k] = 1.0;
        continue;
      }
      if (k >= g->n[ax]) {  // padding column: stays exactly zero
        lam[k] = 1.0;
        continue;
      }
      lam[k] = lam1d(g->N[ax], g->h[ax], k + 1);
      w[k] = (g->load == EIFE_LOAD_LUMPED) ? g->h[ax] / lamA1d(g->N[ax], g->h[ax], k + 1) : 1.0;
      if (g->phi_ready) {
        const double z = -g->tau * g->D * lam[k];
        M[k] = std::expm1(z);
        Q[k] = expm1_minus_z(z);
        Mc[k] = std::expm1(g->c2 * z);
      }
    }
    HIP_TRY(hipMemcpy(g->tab[ax], buf.data(), buf.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  return EIFE_OK;
}

Diag make_diag(const eife_grid_s* g) {
  Diag dg;
  for (int ax = 0; ax < 3; ++ax) {
    const int len = g->tablen[ax];
    dg.ax[ax].lam = g->tab[ax];
    dg.ax[ax].w = g->tab[ax] + len;
    dg.ax[ax].M = g->tab[ax] + 2 * len;
    dg.ax[ax].Q = g->tab[ax] + 3 * len;
    dg.ax[ax].Mc = g->tab[ax] + 4 * len;
  }
  dg.D = g->D;
  dg.tau = g->tau;
  dg.c2 = g->c2;
  return dg;
}

Forcing make_forcing(const eife_grid_s* g, int kind, double t) {
  Forcing F;
  F.kind = kind;
  F.d = g->d;
  F.t = t;
  F.c0 = g->c0;
  F.c1 = g->c1;
  F.D = g->D;
  for (int a = 0; a < 3; ++a) {
    F.a[a] = g->a[a];
    F.h[a] = g->h[a];
  }
  return F;
}

template <typename T>
int set_lds_attrs(size_t bytes) {
  if (bytes <= 65536) return EIFE_OK;
  const int b = int(bytes);
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&row_pass<T, ROW_PHYS>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, b));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&row_pass<T, ROW_FWD_USER>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, b));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&row_pass<T, ROW_INV_USER>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, b));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&col_pass<T, COL_PLAIN>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, b));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&col_pass<T, COL_STAGE_A>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, b));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&col_pass<T, COL_STAGE_B>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, b));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&col_pass<T, COL_ETD1>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, b));
  return EIFE_OK;
}

hipEvent_t take_event(eife_grid_s* g) {
  if (!g->ev_pool.empty()) {
    hipEvent_t e = g->ev_pool.back();
    g->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records the start event of a pass when profiling; returns the pending index or -1.
int prof_begin(eife_grid_s* g, int kind, hipStream_t s) {
  if (!g->prof_on) return -1;
  hipEvent_t a = take_event(g), b = take_event(g);
  if (!a || !b) return -1;
  if (hipEventRecord(a, s) != hipSuccess) return -1;
  g->prof_pending.push_back({kind, a, b});
  return int(g->prof_pending.size()) - 1;
}

void prof_end(eife_grid_s* g, int idx, hipStream_t s) {
  if (idx < 0) return;
  (void)hipEventRecord(g->prof_pending[idx].b, s);
}

int prof_collect(eife_grid_s* g) {
  for (auto& r : g->prof_pending) {
    HIP_TRY(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    g->prof_ms[r.kind] += ms;
    g->prof_n[r.kind] += 1;
    g->ev_pool.push_back(r.a);
    g->ev_pool.push_back(r.b);
  }
  g->prof_pending.clear();
  return EIFE_OK;
}

// Line pairs per block of the fast passes (LDS <= 64 KB, 64-byte column segments).
template <typename T, int L>
constexpr int fast_pb() {
  return sizeof(T) == 4 ? (L == 128 ? 16 : (L == 1024 ? 4 : 8)) : (L == 128 ? 8 : (L == 1024 ? 2 : 4));
}

bool fast_len(int N) { return N == 64 || N == 128 || N == 256 || N == 512; }

template <typename T, int L>
void row_fast_launch(int mode, int nrows, hipStream_t s, const T* src, T* dst, T* dst2, const RowGeom& rg,
                     const Cx<T>* tw, const Forcing& F) {
  constexpr int PB = fast_pb<T, L>();
  constexpr int NT = PB * fast::FftShape<L>::LP;
  dim3 grid((nrows + 2 * PB - 1) / (2 * PB));
  if (mode == ROW_PHYS) {
    if (F.kind == FK_AC)
      hipLaunchKernelGGL((fast::row_fast<T, L, PB, ROW_PHYS, fast::RK_AC>), grid, dim3(NT), 0, s, src, dst, dst2,
                         rg, tw, F);
    else
      hipLaunchKernelGGL((fast::row_fast<T, L, PB, ROW_PHYS, fast::RK_GENERIC>), grid, dim3(NT), 0, s, src, dst,
                         dst2, rg, tw, F);
  } else if (mode == ROW_FWD_USER) {
    hipLaunchKernelGGL((fast::row_fast<T, L, PB, ROW_FWD_USER, fast::RK_GENERIC>), grid, dim3(NT), 0, s, src, dst,
                       dst2, rg, tw, F);
  } else {
    hipLaunchKernelGGL((fast::row_fast<T, L, PB, ROW_INV_USER, fast::RK_GENERIC>), grid, dim3(NT), 0, s, src, dst,
                       dst2, rg, tw, F);
  }
}

// Column passes: 128-byte row segments (32 FP32 / 16 FP64 columns); pairs per
// wavefront slice chosen so a block has at most 512 threads.
template <typename T, int L>
constexpr int col_pb() {
  return (L >= 1024) ? (sizeof(T) == 4 ? 8 : 4) : (sizeof(T) == 4 ? 16 : 8);
}
template <typename T, int L>
constexpr int col_ppw() {
  return (col_pb<T, L>() * fast::FftShape<L>::LP > 512) ? col_pb<T, L>() * fast::FftShape<L>::LP / 512 : 1;
}

template <typename T, int L>
void col_fast_launch(int mode, int pitch, int outer, hipStream_t s, T* W, T* H, const ColGeom& cg,
                     const Cx<T>* tw, const Diag& dg) {
  constexpr int PB = col_pb<T, L>();
  constexpr int PPW = col_ppw<T, L>();
  constexpr int NT = PB / PPW * fast::FftShape<L>::LP;
  dim3 grid(pitch / (2 * PB), outer);
  if (mode == COL_PLAIN) {
    const int ntx = pitch / (2 * PB);
    const int ntiles = ntx * outer;
    constexpr int lds = PB * fast::FftShape<L>::BUF * int(sizeof(Cx<T>));
    constexpr int per_cu = std::max(1, std::min(kPipeBlocksPerCu, 160 * 1024 / lds));
    const int nblk = std::min(ntiles, g_cus * per_cu);
    hipLaunchKernelGGL((fast::col_pipe<T, L, PB, PPW>), dim3(nblk), dim3(NT), 0, s, W, cg, tw, ntx, ntiles);
  } else if (mode == COL_STAGE_A)
    hipLaunchKernelGGL((fast::col_fast<T, L, PB, PPW, COL_STAGE_A>), grid, dim3(NT), 0, s, W, H, cg, tw, dg);
  else if (mode == COL_STAGE_B)
    hipLaunchKernelGGL((fast::col_fast<T, L, PB, PPW, COL_STAGE_B>), grid, dim3(NT), 0, s, W, H, cg, tw, dg);
  else
    hipLaunchKernelGGL((fast::col_fast<T, L, PB, PPW, COL_ETD1>), grid, dim3(NT), 0, s, W, H, cg, tw, dg);
}

template <typename T>
bool try_row_fast(const eife_grid_s* g, int mode, hipStream_t s, const T* src, T* dst, T* dst2, const RowGeom& rg,
                  const Cx<T>* tw, const Forcing& F) {
  if (g->transform != EIFE_TX_FFT || !fast_len(g->N[0])) return false;
  switch (g->N[0]) {
    case 64: row_fast_launch<T, 128>(mode, rg.nrows, s, src, dst, dst2, rg, tw, F); return true;
    case 128: row_fast_launch<T, 256>(mode, rg.nrows, s, src, dst, dst2, rg, tw, F); return true;
    case 256: row_fast_launch<T, 512>(mode, rg.nrows, s, src, dst, dst2, rg, tw, F); return true;
    case 512: row_fast_launch<T, 1024>(mode, rg.nrows, s, src, dst, dst2, rg, tw, F); return true;
  }
  return false;
}

template <typename T>
bool try_col_fast(const eife_grid_s* g, int axis, int mode, int outer, hipStream_t s, T* W, T* H,
                  const ColGeom& cg, const Cx<T>* tw, const Diag& dg) {
  if (g->transform != EIFE_TX_FFT || !fast_len(g->N[axis])) return false;
  switch (g->N[axis]) {
    case 64: col_fast_launch<T, 128>(mode, g->pitch, outer, s, W, H, cg, tw, dg); return true;
    case 128: col_fast_launch<T, 256>(mode, g->pitch, outer, s, W, H, cg, tw, dg); return true;
    case 256: col_fast_launch<T, 512>(mode, g->pitch, outer, s, W, H, cg, tw, dg); return true;
    case 512: col_fast_launch<T, 1024>(mode, g->pitch, outer, s, W, H, cg, tw, dg); return true;
  }
  return false;
}

template <typename T>
int launch_row(eife_grid_s* g, int mode, const T* src, int64_t ld_src, T* dst, int64_t ld_dst, T* dst2,
               const Forcing& F, hipStream_t s) {
  RowGeom rg;
  rg.n = g->n[0];
  rg.nrows = g->nlines_total();
  rg.ny = g->n[1];
  rg.ld_src = ld_src;
  rg.ld_dst = ld_dst;
  rg.pl = g->plan[0];
  rg.P = g->prow;
  rg.ls = rg.pl.L + 1;
  const size_t shm = lds_bytes(g, rg.P, rg.pl.L);
  dim3 grid((rg.nrows + 2 * rg.P - 1) / (2 * rg.P));
  const Cx<T>* tw = reinterpret_cast<const Cx<T>*>(g->tw[0]);
  const int pidx = prof_begin(g, mode == ROW_PHYS ? EIFE_PASS_ROW_PHYS
                                 : mode == ROW_FWD_USER ? EIFE_PASS_ROW_FWD : EIFE_PASS_ROW_INV, s);
  if (try_row_fast<T>(g, mode, s, src, dst, dst2, rg, tw, F)) {
    HIP_TRY(hipGetLastError());
    prof_end(g, pidx, s);
    return EIFE_OK;
  }
  switch (mode) {
    case ROW_PHYS:
      hipLaunchKernelGGL((row_pass<T, ROW_PHYS>), grid, dim3(kThreads), shm, s, src, dst, dst2, rg, tw, F);
      break;
    case ROW_FWD_USER:
      hipLaunchKernelGGL((row_pass<T, ROW_FWD_USER>), grid, dim3(kThreads), shm, s, src, dst, dst2, rg, tw, F);
      break;
    default:
      hipLaunchKernelGGL((row_pass<T, ROW_INV_USER>), grid, dim3(kThreads), shm, s, src, dst, dst2, rg, tw, F);
      break;
  }
  HIP_TRY(hipGetLastError());
  prof_end(g, pidx, s);
  return EIFE_OK;
}

// axis = 1 (y) or 2 (z); `last` selects the diagonal mode
template <typename T>
int launch_col(eife_grid_s* g, int axis, int mode, T* W, T* H, const Diag& dg, hipStream_t s) {
  ColGeom cg;
  const int64_t pitch = g->pitch;
  int outer;
  if (axis == 1) {
    cg.n = g->n[1];
    cg.ld_line = pitch;
    cg.ld_outer = pitch * g->n[1];
    outer = g->n[2];
    cg.last_is_z = 0;
  } else {
    cg.n = g->n[2];
    cg.ld_line = pitch * g->n[1];
    cg.ld_outer = pitch;
    outer = g->n[1];
    cg.last_is_z = 1;
  }
  cg.pl = g->plan[axis];
  cg.P = g->pcol[axis];
  cg.ls = cg.pl.L + 1;
  const size_t shm = lds_bytes(g, cg.P, cg.pl.L);
  dim3 grid(g->pitch / (2 * cg.P), outer);
  const Cx<T>* tw = reinterpret_cast<const Cx<T>*>(g->tw[axis]);
  int kind = EIFE_PASS_MID;
  if (!(axis == 1 && g->d == 3)) {
    kind = mode == COL_PLAIN ? EIFE_PASS_LAST_PLAIN
           : mode == COL_STAGE_A ? EIFE_PASS_LAST_A
           : mode == COL_STAGE_B ? EIFE_PASS_LAST_B : EIFE_PASS_LAST_ETD1;
  }
  const int pidx = prof_begin(g, kind, s);
  if (try_col_fast<T>(g, axis, mode, outer, s, W, H, cg, tw, dg)) {
    HIP_TRY(hipGetLastError());
    prof_end(g, pidx, s);
    return EIFE_OK;
  }
  switch (mode) {
    case COL_PLAIN:
      hipLaunchKernelGGL((col_pass<T, COL_PLAIN>), grid, dim3(kThreads), shm, s, W, H, cg, tw, dg);
      break;
    case COL_STAGE_A:
      hipLaunchKernelGGL((col_pass<T, COL_STAGE_A>), grid, dim3(kThreads), shm, s, W, H, cg, tw, dg);
      break;
    case COL_STAGE_B:
      hipLaunchKernelGGL((col_pass<T, COL_STAGE_B>), grid, dim3(kThreads), shm, s, W, H, cg, tw, dg);
      break;
    default:
      hipLaunchKernelGGL((col_pass<T, COL_ETD1>), grid, dim3(kThreads), shm, s, W, H, cg, tw, dg);
      break;
  }
  HIP_TRY(hipGetLastError());
  prof_end(g, pidx, s);
  return EIFE_OK;
}

#define RET_IF(x)             \
  do {                        \
    int _r = (x);             \
    if (_r != EIFE_OK) return _r; \
  } while (0)

template <typename T>
int run_steps(eife_grid_s* g, T* u, int64_t n_steps, int f_kind, double t0, hipStream_t s) {
  T* W = static_cast<T*>(g->W);
  T* H = static_cast<T*>(g->H);
  const Diag dg = make_diag(g);
  const bool three = g->d == 3;
  const int last = three ? 2 : 1;
  const Forcing F0 = make_forcing(g, f_kind, t0);
  // prologue: W = S_x u, H = S u
  RET_IF(launch_row<T>(g, ROW_FWD_USER, u, g->n[0], W, g->pitch, H, F0, s));
  if (three) RET_IF(launch_col<T>(g, 1, COL_PLAIN, H, H, dg, s));
  RET_IF(launch_col<T>(g, last, COL_PLAIN, H, H, dg, s));
  for (int64_t st = 0; st < n_steps; ++st) {
    const double tn = t0 + double(st) * g->tau;
    RET_IF(launch_row<T>(g, ROW_PHYS, W, g->pitch, W, g->pitch, nullptr, make_forcing(g, f_kind, tn), s));
    if (three) RET_IF(launch_col<T>(g, 1, COL_PLAIN, W, H, dg, s));
    RET_IF(launch_col<T>(g, last, g->stages == 1 ? COL_ETD1 : COL_STAGE_A, W, H, dg, s));
    if (three) RET_IF(launch_col<T>(g, 1, COL_PLAIN, W, H, dg, s));
    if (g->stages == 2) {
      RET_IF(launch_row<T>(g, ROW_PHYS, W, g->pitch, W, g->pitch, nullptr,
                           make_forcing(g, f_kind, tn + g->c2 * g->tau), s));
      if (three) RET_IF(launch_col<T>(g, 1, COL_PLAIN, W, H, dg, s));
      RET_IF(launch_col<T>(g, last, COL_STAGE_B, W, H, dg, s));
      if (three) RET_IF(launch_col<T>(g, 1, COL_PLAIN, W, H, dg, s));
    }
  }
  // epilogue: u = S_x^{-1} W
  RET_IF(launch_row<T>(g, ROW_INV_USER, W, g->pitch, u, g->n[0], nullptr, F0, s));
  return EIFE_OK;
}

NormGeom make_norm_geom(const eife_grid_s* g) {
  NormGeom ng;
  ng.d = g->d;
  ng.cellvol = 1.0;
  for (int a = 0; a < 3; ++a) {
    ng.n[a] = g->n[a];
    if (a < g->d) {
      const double h = g->h[a];
      ng.ad[a] = 4.0 * h / 6.0;
      ng.ao[a] = h / 6.0;
      ng.bd[a] = 2.0 / h;
      ng.bo[a] = -1.0 / h;
      ng.cellvol *= h;
    } else {
      ng.ad[a] = 1.0;
      ng.ao[a] = 0.0;
      ng.bd[a] = 0.0;
      ng.bo[a] = 0.0;
    }
  }
  return ng;
}

template <typename T>
int run_norms(eife_grid_s* g, const void* u, const void* uref, hipStream_t s) {
  const NormGeom ng = make_norm_geom(g);
  const int64_t total = int64_t(g->n[0]) * g->n[1] * g->n[2];
  int nb = int(std::min<int64_t>(kNormBlocksMax, (total + kNormThreads - 1) / kNormThreads));
  nb = std::max(nb, 1);
  hipLaunchKernelGGL((norm_partial<T>), dim3(nb), dim3(kNormThreads), 0, s, static_cast<const T*>(u),
                     static_cast<const T*>(uref), ng, g->partials);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(norm_final, dim3(1), dim3(kNormAcc), 0, s, g->partials, nb, g->out5);
  HIP_TRY(hipGetLastError());
  return EIFE_OK;
}

int check_grid(eife_grid g) {
  if (!g) return fail(EIFE_EINVAL, "null grid");
  return EIFE_OK;
}

void free_grid(eife_grid_s* g) {
  if (!g) return;
  hipFree(g->W);
  hipFree(g->H);
  for (int a = 0; a < 3; ++a) {
    hipFree(g->tw[a]);
    hipFree(g->tab[a]);
  }
  for (auto& r : g->prof_pending) {
    g->ev_pool.push_back(r.a);
    g->ev_pool.push_back(r.b);
  }
  for (hipEvent_t e : g->ev_pool) hipEventDestroy(e);
  hipFree(g->partials);
  hipFree(g->out5);
  if (g->host5) hipHostFree(g->host5);
  delete g;
}

}  // namespace

extern "C" {

int eife_version(void) { return 1; }

const char* eife_last_error(void) { return g_last_error.c_str(); }

int eife_create_grid(int d, const int32_t* N, const double* h, double D, int bc, int dtype, eife_grid* out) {
  if (!out) return fail(EIFE_EINVAL, "out is null");
  *out = nullptr;
  if (d < 1 || d > 3) return fail(EIFE_EINVAL, "d must be 1, 2 or 3 (got %d)", d);
  if (!N || !h) return fail(EIFE_EINVAL, "N and h must not be null");
  if (!(D > 0.0) || !std::isfinite(D)) return fail(EIFE_EINVAL, "D must be a positive finite number");
  if (bc == EIFE_BC_PERIODIC) return fail(EIFE_EUNSUPPORTED, "periodic boundary conditions are not implemented");
  if (bc != EIFE_BC_DIRICHLET) return fail(EIFE_EINVAL, "unknown boundary condition %d", bc);
  if (dtype != EIFE_F32 && dtype != EIFE_F64) return fail(EIFE_EINVAL, "unknown dtype %d", dtype);
  eife_grid_s* g = new eife_grid_s();
  g->d = d;
  g->dtype = dtype;
  g->esz = dtype == EIFE_F32 ? 4 : 8;
  g->D = D;
  for (int a = 0; a < d; ++a) {
    if (N[a] < 2) {
      delete g;
      return fail(EIFE_EINVAL, "N[%d] = %d must be >= 2", a, N[a]);
    }
    if (N[a] > 4096) {
      delete g;
      return fail(EIFE_EUNSUPPORTED, "N[%d] = %d exceeds 4096", a, N[a]);
    }
    if (!(h[a] > 0.0) || !std::isfinite(h[a])) {
      delete g;
      return fail(EIFE_EINVAL, "h[%d] must be a positive finite number", a);
    }
    g->N[a] = N[a];
    g->n[a] = N[a] - 1;
    g->h[a] = h[a];
  }
  for (int a = 0; a < 3; ++a) {
    if (!factor_plan(2 * g->N[a], &g->plan[a])) {
      const int bad = g->N[a];
      delete g;
      return fail(EIFE_EUNSUPPORTED, "N = %d is not of the form 2^i 3^j", bad);
    }
  }
  g->pitch = ((g->n[0] + 31) / 32) * 32;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    delete g;
    return fail(EIFE_EHIP, "no HIP device");
  }
  g->device = dev;
  int maxlds = 65536;
  if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) maxlds = 65536;
  g->max_lds = size_t(maxlds);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) g_cus = cus;
  // launch shapes
  g->prow = pick_pairs(g, g->plan[0].L, std::min(16, (g->nlines_total() + 1) / 2));
  for (int a = 1; a < 3; ++a) {
    int P = pick_pairs(g, g->plan[a].L, 16);
    while (g->pitch % (2 * P) != 0) P--;
    g->pcol[a] = P;
  }
  size_t need = lds_bytes(g, g->prow, g->plan[0].L);
  for (int a = 1; a < 3; ++a) need = std::max(need, lds_bytes(g, g->pcol[a], g->plan[a].L));
  if (need > g->max_lds) {
    free_grid(g);
    return fail(EIFE_EUNSUPPORTED, "a line of this grid needs %zu bytes of LDS, device allows %zu", need,
                g->max_lds);
  }
  const int r = dtype == EIFE_F32 ? set_lds_attrs<float>(need) : set_lds_attrs<double>(need);
  if (r != EIFE_OK) {
    free_grid(g);
    return r;
  }
  const size_t elems = size_t(g->pitch) * g->n[1] * g->n[2];
  if (hipMalloc(&g->W, elems * g->esz) != hipSuccess || hipMalloc(&g->H, elems * g->esz) != hipSuccess) {
    free_grid(g);
    return fail(EIFE_ENOMEM, "cannot allocate %zu bytes of workspace", 2 * elems * g->esz);
  }
  if (hipMemset(g->W, 0, elems * g->esz) != hipSuccess || hipMemset(g->H, 0, elems * g->esz) != hipSuccess) {
    free_grid(g);
    return fail(EIFE_EHIP, "hipMemset failed");
  }
  for (int a = 0; a < 3; ++a) {
    const int L = g->plan[a].L;
    size_t bytes;
    if (dtype == EIFE_F32) {
      std::vector<Cx<float>> v;
      fill_twiddles(v, L);
      bytes = v.size() * sizeof(v[0]);
      if (hipMalloc(&g->tw[a], bytes) != hipSuccess ||
          hipMemcpy(g->tw[a], v.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        free_grid(g);
        return fail(EIFE_ENOMEM, "twiddle table allocation failed");
      }
    } else {
      std::vector<Cx<double>> v;
      fill_twiddles(v, L);
      bytes = v.size() * sizeof(v[0]);
      if (hipMalloc(&g->tw[a], bytes) != hipSuccess ||
          hipMemcpy(g->tw[a], v.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        free_grid(g);
        return fail(EIFE_ENOMEM, "twiddle table allocation failed");
      }
    }
    g->tablen[a] = (a == 0) ? g->pitch : g->n[a];
    if (hipMalloc(reinterpret_cast<void**>(&g->tab[a]), kTabArrays * size_t(g->tablen[a]) * sizeof(double)) != hipSuccess) {
      free_grid(g);
      return fail(EIFE_ENOMEM, "table allocation failed");
    }
  }
  if (hipMalloc(reinterpret_cast<void**>(&g->partials), kNormBlocksMax * kNormAcc * sizeof(double)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&g->out5), kNormAcc * sizeof(double)) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&g->host5), kNormAcc * sizeof(double), 0) != hipSuccess) {
    free_grid(g);
    return fail(EIFE_ENOMEM, "norm buffers allocation failed");
  }
  const int rt = upload_tables(g);
  if (rt != EIFE_OK) {
    free_grid(g);
    return rt;
  }
  *out = g;
  return EIFE_OK;
}

int eife_destroy_grid(eife_grid g) {
  free_grid(g);
  return EIFE_OK;
}

int eife_set_c2(eife_grid g, double c2) {
  RET_IF(check_grid(g));
  if (!(c2 > 0.0 && c2 <= 1.0)) return fail(EIFE_EINVAL, "c2 must lie in (0, 1]");
  g->c2 = c2;
  g->phi_ready = false;
  return EIFE_OK;
}

int eife_set_origin(eife_grid g, const double* a) {
  RET_IF(check_grid(g));
  if (!a) return fail(EIFE_EINVAL, "origin is null");
  for (int i = 0; i < g->d; ++i) {
    if (!std::isfinite(a[i])) return fail(EIFE_EINVAL, "origin must be finite");
    g->a[i] = a[i];
  }
  return EIFE_OK;
}

int eife_set_load(eife_grid g, int kind) {
  RET_IF(check_grid(g));
  if (kind != EIFE_LOAD_LUMPED && kind != EIFE_LOAD_NODAL) return fail(EIFE_EINVAL, "unknown load kind %d", kind);
  g->load = kind;
  return upload_tables(g);
}

int eife_set_transform(eife_grid g, int kind) {
  RET_IF(check_grid(g));
  if (kind == EIFE_TX_GEMM_SPLITBF16) return fail(EIFE_EUNSUPPORTED, "the split-BF16 GEMM transform is not built");
  if (kind != EIFE_TX_FFT && kind != EIFE_TX_FFT_GENERIC) return fail(EIFE_EINVAL, "unknown transform kind %d", kind);
  g->transform = kind;
  return EIFE_OK;
}

int eife_set_forcing(eife_grid g, double c0, double c1) {
  RET_IF(check_grid(g));
  if (!std::isfinite(c0) || !std::isfinite(c1)) return fail(EIFE_EINVAL, "forcing parameters must be finite");
  g->c0 = c0;
  g->c1 = c1;
  return EIFE_OK;
}

int eife_set_phi(eife_grid g, double tau, int stages) {
  RET_IF(check_grid(g));
  if (!(tau > 0.0) || !std::isfinite(tau)) return fail(EIFE_EINVAL, "tau must be a positive finite number");
  if (stages != 1 && stages != 2) return fail(EIFE_EINVAL, "stages must be 1 or 2 (got %d)", stages);
  g->tau = tau;
  g->stages = stages;
  g->phi_ready = true;
  const int r = upload_tables(g);
  if (r != EIFE_OK) g->phi_ready = false;
  return r;
}

int eife_profile(eife_grid g, int on) {
  RET_IF(check_grid(g));
  RET_IF(prof_collect(g));
  for (int k = 0; k < EIFE_PASS_COUNT; ++k) {
    g->prof_ms[k] = 0.0;
    g->prof_n[k] = 0;
  }
  g->prof_on = on != 0;
  return EIFE_OK;
}

int eife_profile_read(eife_grid g, double* ms, int64_t* launches) {
  RET_IF(check_grid(g));
  if (!ms || !launches) return fail(EIFE_EINVAL, "ms and launches must not be null");
  RET_IF(prof_collect(g));
  for (int k = 0; k < EIFE_PASS_COUNT; ++k) {
    ms[k] = g->prof_ms[k];
    launches[k] = g->prof_n[k];
  }
  return EIFE_OK;
}

int eife_grid_size(eife_grid g, int64_t* count) {
  RET_IF(check_grid(g));
  if (!count) return fail(EIFE_EINVAL, "count is null");
  *count = int64_t(g->n[0]) * g->n[1] * g->n[2];
  return EIFE_OK;
}

int eife_step(eife_grid g, void* u, int64_t n_steps, int f_kind, double t0, void* stream) {
  RET_IF(check_grid(g));
  if (!u) return fail(EIFE_EINVAL, "u is null");
  if (n_steps < 0) return fail(EIFE_EINVAL, "n_steps must be >= 0");
  if (f_kind < EIFE_F_ZERO || f_kind > EIFE_F_AFFINE_T) return fail(EIFE_EINVAL, "unknown f_kind %d", f_kind);
  if (f_kind == EIFE_F_EX51 && g->d != 2) return fail(EIFE_EINVAL, "EIFE_F_EX51 is a 2D problem");
  if (!std::isfinite(t0)) return fail(EIFE_EINVAL, "t0 must be finite");
  if (!g->phi_ready) return fail(EIFE_ESTATE, "eife_set_phi must be called before eife_step");
  if (n_steps == 0) return EIFE_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (g->dtype == EIFE_F32) return run_steps<float>(g, static_cast<float*>(u), n_steps, f_kind, t0, s);
  return run_steps<double>(g, static_cast<double*>(u), n_steps, f_kind, t0, s);
}

int eife_norms(eife_grid g, const void* u, const void* uref, double* out, void* stream) {
  RET_IF(check_grid(g));
  if (!u || !out) return fail(EIFE_EINVAL, "u and out must not be null");
  hipStream_t s = static_cast<hipStream_t>(stream);
  RET_IF(g->dtype == EIFE_F32 ? run_norms<float>(g, u, uref, s) : run_norms<double>(g, u, uref, s));
  HIP_TRY(hipMemcpyAsync(g->host5, g->out5, kNormAcc * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const double* r = g->host5;
  double cellvol = 1.0;
  for (int a = 0; a < g->d; ++a) cellvol *= g->h[a];
  out[0] = std::sqrt(std::max(r[0], 0.0));
  out[1] = std::sqrt(std::max(r[0] + r[1], 0.0));
  out[2] = r[2];
  out[3] = 0.5 * g->D * r[3] + cellvol * r[4];
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(out[k])) return fail(EIFE_ENONFINITE, "norm %d is not finite", k);
  return EIFE_OK;
}

}  // extern "C"

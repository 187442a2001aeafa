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
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/eife.h"
#include "eife_internal.h"
#include "eife_kernels.hpp"
#include "eife_fast.hpp"
#include "eife_gemm.hpp"

// Kernel arguments are passed by value; every pass's argument block (the
// geometry, forcing and diagonal structs plus at most eight pointers and ints)
// stays far below the 4 KB kernel-argument segment.
static_assert(sizeof(eife::RowGeom) + sizeof(eife::Forcing) + 8 * sizeof(void*) <= 1024, "row pass arguments");
static_assert(sizeof(eife::ColGeom) + sizeof(eife::Diag) + 8 * sizeof(void*) <= 1024, "column pass arguments");
static_assert(sizeof(eife::NormGeom) + 8 * sizeof(void*) <= 1024, "norm pass arguments");
#include "eife_long.hpp"

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
// Generic FP64 passes over lines of at least kLongLine FFT points (one or two
// lines fill a block's LDS) run kLongThreads threads per block: more waves per
// compute unit and 8 instead of 32 values per thread.
constexpr int kLongLine = 4096;
constexpr int kLongThreads = 1024;
// FP64 only: FP32 long lines measured slower with the larger blocks (two
// 256-thread blocks of one FP32 line each share a compute unit instead).
template <typename T>
bool long_lines(int L) {
  return sizeof(T) == 8 && L >= kLongLine;
}
constexpr size_t kLdsBudget = 80 * 1024;  // per block, two blocks per CU fit in 160 KB
constexpr int kNormBlocksMax = 8192;
constexpr int kTabArrays = 8;  // lam, w, M, Q, Mc, R, Mc3, Qc3 per axis
constexpr int kPipeBlocksPerCu = 4;  // resident blocks of the pipelined column pass (LDS permitting)
constexpr int kStagePipeMinTiles = 2;  // tiles per resident block from which the stage pass is pipelined
int g_cus = 256;                     // compute units of the device (set at grid creation)

bool factor_plan(int L, FftPlan* pl) {
  pl->L = L;
  pl->n8 = pl->n4 = pl->n2 = pl->n3 = pl->n5 = pl->n7 = pl->nd = 0;
  pl->dr[0] = pl->dr[1] = pl->dr[2] = 0;
  int r = L;
  while (r % 8 == 0) {
    r /= 8;
    pl->n8++;
  }
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
  while (r % 5 == 0) {
    r /= 5;
    pl->n5++;
  }
  while (r % 7 == 0) {
    r /= 7;
    pl->n7++;
  }
  // the remaining prime factors (all above 7) run as direct-DFT stages
  for (int p = 11; p <= r; p += 2) {
    while (r % p == 0) {
      if (pl->nd == 3) return false;
      pl->dr[pl->nd++] = p;
      r /= p;
    }
  }
  return r == 1;
}

}  // namespace

struct eife_grid_s {
  int d = 0;
  int N[3] = {2, 2, 2};
  int n[3] = {1, 1, 1};  // unknowns per axis: N - 1 (Dirichlet), N (periodic); virtual axes: 1
  bool per[3] = {false, false, false};  // periodic axis (real axes of a periodic grid)
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
  double c2_3 = 1.0 / 3.0, c3_3 = 2.0 / 3.0;  // nodes of the three-stage scheme
  void* X = nullptr;  // extra spectral state of the three-stage scheme (allocated on first use)
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
  double* sinpi_ax[3] = {nullptr, nullptr, nullptr};  // sin(pi x) at the interior nodes of each axis
  int tablen[3] = {0, 0, 0};
  double* partials = nullptr;
  double* out5 = nullptr;
  double* host5 = nullptr;  // pinned
  // per-step phi tables of variable-step runs (eife_step_variable): a chunk of
  // steps at a time, each step 3 arrays (M, Q, Mc) per axis
  // (two chunk buffers, filled alternately)
  double* vtab = nullptr;
  double* vhost = nullptr;  // pinned staging copies
  hipEvent_t vev[2] = {nullptr, nullptr};  // copy of the buffer's last chunk done
  int64_t vchunk = 0;       // steps per chunk (0: not allocated)
  std::vector<double> hlam[3];  // host copy of the lambda table of each axis
  // launch shapes
  FftPlan plan[3];
  int transform = EIFE_TX_FFT;
  void* smat[3] = {nullptr, nullptr, nullptr};  // split-BF16 sine matrices (hi then lo, kp x kp each)
  int kp[3] = {0, 0, 0};
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

// expm1(z) - z - z^2/2 for z <= 0: power series below |z| = 1, else direct.
double expm1_minus_z2(double z) {
  if (std::fabs(z) < 1.0) {
    double term = z * z * z / 6.0, sum = 0.0;
    for (int m = 3; m < 60 && term != 0.0; ++m) {
      sum += term;
      term *= z / double(m + 1);
    }
    return sum;
  }
  return std::expm1(z) - z - 0.5 * z * z;
}

// Second node of the scheme in use (the three-stage scheme has its own pair).
double node_c2(const eife_grid_s* g) { return g->stages == 3 ? g->c2_3 : g->c2; }

constexpr int kStepArrays = 6;  // M, Q, Mc, R, Mc3, Qc3

// The step-dependent tables of one axis for step size tau (zeros on virtual
// axes and padding columns, which the stage never reads as nonzero; R, Mc3,
// Qc3 only for the three-stage scheme).  t points at kStepArrays arrays of
// the axis length.
void fill_phi(const eife_grid_s* g, int ax, double tau, double* t) {
  const int len = g->tablen[ax];
  double *M = t, *Q = t + len, *Mc = t + 2 * len, *R = t + 3 * len, *Mc3 = t + 4 * len, *Qc3 = t + 5 * len;
  const double c2 = node_c2(g), c3 = g->c3_3;
  const bool three = g->stages == 3;
  for (int k = 0; k < len; ++k) {
    M[k] = Q[k] = Mc[k] = R[k] = Mc3[k] = Qc3[k] = 0.0;
    if (ax >= g->d || k >= g->n[ax]) continue;
    const double z = -tau * g->D * g->hlam[ax][k];
    M[k] = std::expm1(z);
    Q[k] = expm1_minus_z(z);
    Mc[k] = std::expm1(c2 * z);
    if (three) {
      R[k] = expm1_minus_z2(z);
      Mc3[k] = std::expm1(c3 * z);
      Qc3[k] = expm1_minus_z(c3 * z);
    }
  }
}

int64_t step_table_stride(const eife_grid_s* g) {
  return kStepArrays * (int64_t(g->tablen[0]) + g->tablen[1] + g->tablen[2]);
}

int upload_tables(eife_grid_s* g) {
  for (int ax = 0; ax < 3; ++ax) {
    const int len = g->tablen[ax];
    std::vector<double> buf(kTabArrays * size_t(len), 0.0);
    double* lam = buf.data();
    double* w = lam + len;
    double* M = w + len;
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
      // sine index k + 1 (angle (k + 1) pi / N); periodic position k (angle 2 k pi / N)
      const int kk = g->per[ax] ? 2 * k : k + 1;
      lam[k] = lam1d(g->N[ax], g->h[ax], kk);
      w[k] = (g->load == EIFE_LOAD_LUMPED) ? g->h[ax] / lamA1d(g->N[ax], g->h[ax], kk) : 1.0;
    }
    g->hlam[ax].assign(lam, lam + len);
    if (g->phi_ready) fill_phi(g, ax, g->tau, M);
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
    dg.ax[ax].R = g->tab[ax] + 5 * len;
    dg.ax[ax].Mc3 = g->tab[ax] + 6 * len;
    dg.ax[ax].Qc3 = g->tab[ax] + 7 * len;
  }
  dg.D = g->D;
  dg.tau = g->tau;
  dg.c2 = node_c2(g);
  dg.c3 = g->c3_3;
  dg.X = g->X;
  return dg;
}

// The stage tables of one step of a variable-step run: lam and w as always,
// M, Q, Mc from the step's block of the chunk table.
Diag make_diag_at(const eife_grid_s* g, const double* block, double tau) {
  Diag dg = make_diag(g);
  for (int ax = 0; ax < 3; ++ax) {
    const int len = g->tablen[ax];
    dg.ax[ax].M = block;
    dg.ax[ax].Q = block + len;
    dg.ax[ax].Mc = block + 2 * len;
    dg.ax[ax].R = block + 3 * len;
    dg.ax[ax].Mc3 = block + 4 * len;
    dg.ax[ax].Qc3 = block + 5 * len;
    block += kStepArrays * len;
  }
  dg.tau = tau;
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
    F.n[a] = g->n[a];
    F.sinpi_ax[a] = g->sinpi_ax[a];
  }
  const double PI2 = 9.8696044010893586188;
  F.et = kind == EIFE_F_EX51 ? std::exp(-PI2 * t) : std::exp(-t);
  return F;
}

// The per-axis sin(pi x) tables at the grid's current origin (device, on the
// null stream after all work on the device; blocks the host).
int upload_sinpi(eife_grid_s* g) {
  HIP_TRY(hipDeviceSynchronize());  // no step in flight still reads the old tables
  for (int a = 0; a < 3; ++a) {
    const int n = g->n[a];
    hipLaunchKernelGGL(sinpi_table, dim3((n + 255) / 256), dim3(256), 0, 0, g->sinpi_ax[a], n, g->a[a], g->h[a]);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipDeviceSynchronize());
  return EIFE_OK;
}

template <typename T, bool BAT>
int set_lds_attrs_v(int b) {
  const void* fns[] = {reinterpret_cast<const void*>(&row_pass<T, ROW_PHYS, BAT>),
                       reinterpret_cast<const void*>(&row_pass<T, ROW_FWD_USER, BAT>),
                       reinterpret_cast<const void*>(&row_pass<T, ROW_INV_USER, BAT>),
                       reinterpret_cast<const void*>(&col_pass<T, COL_PLAIN, BAT>),
                       reinterpret_cast<const void*>(&col_pass<T, COL_STAGE_A, BAT>),
                       reinterpret_cast<const void*>(&col_pass<T, COL_STAGE_B, BAT>),
                       reinterpret_cast<const void*>(&col_pass<T, COL_ETD1, BAT>)};
  for (const void* f : fns) HIP_TRY(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, b));
  return EIFE_OK;
}

template <typename T>
int set_lds_attrs(size_t bytes) {
  if (bytes <= 65536) return EIFE_OK;
  const int r = set_lds_attrs_v<T, false>(int(bytes));
  if (r != EIFE_OK) return r;
  return set_lds_attrs_v<T, true>(int(bytes));
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

// ---------------------------------------------------------------------------
// Launch layer.  Every pass launch may cover several instances of one size
// class (a batch): `count` instances, per-instance pointers and tables in
// the device tables `rinst` / `cinst` (null for a single grid).  `var`
// selects a launch shape (pairs per block) among the tuned variants.

// Pairs per block of the specialised kernels: the largest power of two whose
// LDS regions fit the budget (64 KB rows, 80 KB columns = two blocks per CU),
// capped so row blocks stay within 512 threads and column tiles at 128-byte
// row segments.  Variant 1 halves it.
template <typename T, int L>
constexpr int pb_fit(int budget, int cap) {
  int pb = 1;
  while (pb < cap && size_t(2 * pb) * fast::Line<T, L>::BUF * sizeof(Cx<T>) <= size_t(budget)) pb *= 2;
  return pb;
}
template <typename T, int L>
constexpr int row_pb(int var) {
  constexpr int cap = std::min(16, 512 / fast::Line<T, L>::LP);
  constexpr int pb = pb_fit<T, L>(65536, cap);
  return var == 0 ? pb : std::max(1, pb / 2);
}
template <typename T, int L>
constexpr int col_pb(int var) {
  constexpr int pb = pb_fit<T, L>(81920, int(128 / (2 * sizeof(T))));
  return var == 0 ? pb : std::max(1, pb / 2);
}

template <typename T, int L, int PB>
constexpr int col_ppw() {
  return (PB * fast::Line<T, L>::LP > 512) ? PB * fast::Line<T, L>::LP / 512 : 1;
}

// Line lengths with specialised kernels (the three-subsequence form of
// N = 384 needs more registers than double data allows without spilling).
template <typename T>
bool fast_len(int N) {
  return N == 64 || N == 128 || N == 256 || N == 512 || N == 192 || (N == 384 && sizeof(T) == 4);
}

// Host-side checks of a specialised launch: the argument blocks fit the
// kernel-argument segment, block sizes are within the limits (a block may be a
// fraction of a wavefront: one 16-lane line pair), static LDS fits a workgroup
// (160 KB on gfx950), and the grid is non-empty and within range.  A failed
// check skips the launch and is reported by launch_row / launch_col.
static_assert(3 * sizeof(void*) + sizeof(RowGeom) + sizeof(void*) + sizeof(Forcing) + sizeof(void*) <= 1024,
              "row pass arguments");
static_assert(2 * sizeof(void*) + sizeof(ColGeom) + sizeof(void*) + sizeof(Diag) + sizeof(void*) <= 1024,
              "column pass arguments");
thread_local const char* g_bad_launch = nullptr;

bool launch_shape_ok(dim3 grid, int threads, size_t lds_static) {
  const bool ok = grid.x >= 1 && grid.y >= 1 && grid.z >= 1 && grid.x <= 0x7fffffffu && grid.y <= 65535u &&
                  grid.z <= 65535u && threads >= 1 && threads <= 1024 && lds_static <= 160 * 1024;
  if (!ok) g_bad_launch = "specialised pass launch shape out of range";
  return ok;
}

template <typename T, int L, int PB, bool BAT>
void row_fast_go(int mode, int nrows, int count, hipStream_t s, const T* src, T* dst, T* dst2, const RowGeom& rg,
                 const Cx<T>* tw, const Forcing& F, const RowInst<T>* ri) {
  constexpr int NT = PB * fast::Line<T, L>::LP;
  dim3 grid((nrows + 2 * PB - 1) / (2 * PB), count);
  if (!launch_shape_ok(grid, NT, size_t(PB) * fast::Line<T, L>::BUF * sizeof(Cx<T>))) return;
  if (mode == ROW_PHYS) {
    if (F.kind == FK_AC)
      hipLaunchKernelGGL((fast::row_fast<T, L, PB, ROW_PHYS, fast::RK_AC, BAT>), grid, dim3(NT), 0, s, src, dst,
                         dst2, rg, tw, F, ri);
    else
      hipLaunchKernelGGL((fast::row_fast<T, L, PB, ROW_PHYS, fast::RK_GENERIC, BAT>), grid, dim3(NT), 0, s, src,
                         dst, dst2, rg, tw, F, ri);
  } else if (mode == ROW_FWD_PHYS) {
    if (F.kind == FK_AC)
      hipLaunchKernelGGL((fast::row_fast<T, L, PB, ROW_FWD_PHYS, fast::RK_AC, BAT>), grid, dim3(NT), 0, s, src, dst,
                         dst2, rg, tw, F, ri);
    else
      hipLaunchKernelGGL((fast::row_fast<T, L, PB, ROW_FWD_PHYS, fast::RK_GENERIC, BAT>), grid, dim3(NT), 0, s, src,
                         dst, dst2, rg, tw, F, ri);
  } else if (mode == ROW_FWD_USER) {
    hipLaunchKernelGGL((fast::row_fast<T, L, PB, ROW_FWD_USER, fast::RK_GENERIC, BAT>), grid, dim3(NT), 0, s, src,
                       dst, dst2, rg, tw, F, ri);
  } else if (mode == ROW_INV_CHG) {
    if constexpr (fast::Line<T, L>::LP == 64 && !BAT)
      hipLaunchKernelGGL((fast::row_fast<T, L, PB, ROW_INV_CHG, fast::RK_GENERIC, BAT>), grid, dim3(NT), 0, s, src,
                         dst, dst2, rg, tw, F, ri);
  } else {
    hipLaunchKernelGGL((fast::row_fast<T, L, PB, ROW_INV_USER, fast::RK_GENERIC, BAT>), grid, dim3(NT), 0, s, src,
                       dst, dst2, rg, tw, F, ri);
  }
}

template <typename T, int L>
void row_fast_launch(int var, int mode, int nrows, int count, hipStream_t s, const T* src, T* dst, T* dst2,
                     const RowGeom& rg, const Cx<T>* tw, const Forcing& F, const RowInst<T>* ri) {
  if (ri) {
    if (var == 0)
      row_fast_go<T, L, row_pb<T, L>(0), true>(mode, nrows, count, s, src, dst, dst2, rg, tw, F, ri);
    else
      row_fast_go<T, L, row_pb<T, L>(1), true>(mode, nrows, count, s, src, dst, dst2, rg, tw, F, ri);
  } else {
    // a single grid with few rows (2D grids up to N = 512): fewer pairs per
    // block so that the launch spreads over the compute units
    constexpr int pb0 = row_pb<T, L>(0);
    constexpr int pbs = std::max(1, pb0 / 4);
    if ((nrows + 2 * pb0 - 1) / (2 * pb0) < g_cus)
      row_fast_go<T, L, pbs, false>(mode, nrows, count, s, src, dst, dst2, rg, tw, F, ri);
    else
      row_fast_go<T, L, pb0, false>(mode, nrows, count, s, src, dst, dst2, rg, tw, F, ri);
  }
}

template <typename T, int L, int PB, bool BAT>
void col_fast_go(int mode, int pitch, int outer, int count, bool pipe, hipStream_t s, T* W, T* H, const ColGeom& cg,
                 const Cx<T>* tw, const Diag& dg, const ColInst<T>* ci) {
  constexpr int PPW = col_ppw<T, L, PB>();
  constexpr int NT = PB / PPW * fast::Line<T, L>::LP;
  dim3 grid(pitch / (2 * PB), outer, count);
  if (!launch_shape_ok(grid, NT, size_t(PB) * fast::Line<T, L>::BUF * sizeof(Cx<T>))) return;
  if (mode == COL_PLAIN) {
    // FP32: the persistent pass that prefetches each next tile; FP64 one tile
    // per block (the prefetch registers would leave three waves per SIMD, one
    // block per CU, where one tile per block fits two blocks: measured faster)
    if (pipe && !ci && sizeof(T) == 4) {
      const int ntx = pitch / (2 * PB);
      const int ntiles = ntx * outer;
      constexpr int lds = PB * fast::Line<T, L>::BUF * int(sizeof(Cx<T>));
      constexpr int per_cu = std::max(1, std::min(kPipeBlocksPerCu, 160 * 1024 / lds));
      const int nblk = std::min(ntiles, g_cus * per_cu);
      hipLaunchKernelGGL((fast::col_pipe<T, L, PB, PPW>), dim3(nblk), dim3(NT), 0, s, W, cg, tw, ntx, ntiles);
    } else {
      hipLaunchKernelGGL((fast::col_fast<T, L, PB, PPW, COL_PLAIN, BAT>), grid, dim3(NT), 0, s, W, H, cg, tw, dg, ci);
    }
    return;
  }
  // FP32 power-of-two lines up to 512 points: the persistent pipelined stage
  // pass fits 4 waves per SIMD without spilling; longer, radix-3 or FP64 lines
  // keep one tile per block
  if constexpr (!BAT && sizeof(T) == 4 && fast::IsPow2<L>::value && L <= 512) {
    // many tiles per resident block: the persistent pipelined stage pass
    const int ntx = pitch / (2 * PB);
    const int ntiles = ntx * outer;
    constexpr int lds = PB * fast::Line<T, L>::BUF * int(sizeof(Cx<T>));
    constexpr int per_cu = std::max(1, std::min(kPipeBlocksPerCu, 160 * 1024 / lds));
    const int nblk = g_cus * per_cu;
    if (pipe && ntiles >= kStagePipeMinTiles * nblk && mode < COL_S3_1) {
      if (mode == COL_STAGE_A)
        hipLaunchKernelGGL((fast::col_stage_pipe<T, L, PB, PPW, COL_STAGE_A>), dim3(nblk), dim3(NT), 0, s, W, H, cg,
                           tw, dg, ntx, ntiles, (const ColInst<T>*)nullptr, 0);
      else if (mode == COL_STAGE_B)
        hipLaunchKernelGGL((fast::col_stage_pipe<T, L, PB, PPW, COL_STAGE_B>), dim3(nblk), dim3(NT), 0, s, W, H, cg,
                           tw, dg, ntx, ntiles, (const ColInst<T>*)nullptr, 0);
      else
        hipLaunchKernelGGL((fast::col_stage_pipe<T, L, PB, PPW, COL_ETD1>), dim3(nblk), dim3(NT), 0, s, W, H, cg,
                           tw, dg, ntx, ntiles, (const ColInst<T>*)nullptr, 0);
      return;
    }
  }
  // batched FP32 classes, column variant 2: the pipelined stage pass over
  // every tile of every instance (faster for 1024-point lines, where one
  // 8-wave block fills a CU; slower for 768-point lines: the autotuner decides)
  if constexpr (BAT && sizeof(T) == 4) {
    if (pipe && ci && (mode == COL_STAGE_A || mode == COL_STAGE_B || mode == COL_ETD1)) {
      const int ntx = pitch / (2 * PB);
      const int tpi = ntx * outer;
      const int ntiles = tpi * count;
      auto go = [&](auto kern) {
        static int per_cu = 0;
        if (per_cu == 0 &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), NT, 0) !=
                hipSuccess)
          per_cu = 1;
        const int nblk = std::min(ntiles, g_cus * std::max(1, per_cu));
        if (!launch_shape_ok(dim3(nblk), NT, size_t(PB) * fast::Line<T, L>::BUF * sizeof(Cx<T>))) return;
        hipLaunchKernelGGL(kern, dim3(nblk), dim3(NT), 0, s, W, H, cg, tw, dg, ntx, ntiles, ci, tpi);
      };
      if (mode == COL_STAGE_A)
        go(fast::col_stage_pipe<T, L, PB, PPW, COL_STAGE_A, true>);
      else if (mode == COL_STAGE_B)
        go(fast::col_stage_pipe<T, L, PB, PPW, COL_STAGE_B, true>);
      else
        go(fast::col_stage_pipe<T, L, PB, PPW, COL_ETD1, true>);
      return;
    }
  }
  if constexpr (!BAT) {
    if (mode == COL_S3_1 || mode == COL_S3_2 || mode == COL_S3_3) {
      if (mode == COL_S3_1)
        hipLaunchKernelGGL((fast::col_fast<T, L, PB, PPW, COL_S3_1, false>), grid, dim3(NT), 0, s, W, H, cg, tw, dg, ci);
      else if (mode == COL_S3_2)
        hipLaunchKernelGGL((fast::col_fast<T, L, PB, PPW, COL_S3_2, false>), grid, dim3(NT), 0, s, W, H, cg, tw, dg, ci);
      else
        hipLaunchKernelGGL((fast::col_fast<T, L, PB, PPW, COL_S3_3, false>), grid, dim3(NT), 0, s, W, H, cg, tw, dg, ci);
      return;
    }
  }
  if (mode == COL_STAGE_A) {
    hipLaunchKernelGGL((fast::col_fast<T, L, PB, PPW, COL_STAGE_A, BAT>), grid, dim3(NT), 0, s, W, H, cg, tw, dg, ci);
  } else if (mode == COL_STAGE_B) {
    hipLaunchKernelGGL((fast::col_fast<T, L, PB, PPW, COL_STAGE_B, BAT>), grid, dim3(NT), 0, s, W, H, cg, tw, dg, ci);
  } else {
    hipLaunchKernelGGL((fast::col_fast<T, L, PB, PPW, COL_ETD1, BAT>), grid, dim3(NT), 0, s, W, H, cg, tw, dg, ci);
  }
}

template <typename T, int L>
void col_fast_launch(int var, int mode, int pitch, int outer, int count, hipStream_t s, T* W, T* H,
                     const ColGeom& cg, const Cx<T>* tw, const Diag& dg, const ColInst<T>* ci) {
  if (ci) {
    // batched variants: 0 / 1 the two tile widths (one tile per block), 2 / 3
    // the same widths in the persistent pipelined stage pass
    if (var == 1 || var == 3)
      col_fast_go<T, L, col_pb<T, L>(1), true>(mode, pitch, outer, count, var == 3, s, W, H, cg, tw, dg, ci);
    else
      col_fast_go<T, L, col_pb<T, L>(0), true>(mode, pitch, outer, count, var == 2, s, W, H, cg, tw, dg, ci);
  } else {
    // a single grid with few column tiles (2D grids): narrower tiles
    constexpr int pb0 = col_pb<T, L>(0);
    constexpr int pbs = std::max(1, pb0 / 8);
    if ((pitch / (2 * pb0)) * outer < g_cus)
      col_fast_go<T, L, pbs, false>(mode, pitch, outer, count, true, s, W, H, cg, tw, dg, ci);
    else
      col_fast_go<T, L, pb0, false>(mode, pitch, outer, count, true, s, W, H, cg, tw, dg, ci);
  }
}

// Periodic lines with wave-local kernels: N = L = 128, 256, 512 (single grids).
inline bool per_fast_len(int N) { return N == 128 || N == 256 || N == 512; }

template <typename T, int L>
void row_per_launch(int mode, int nrows, hipStream_t s, const T* src, T* dst, T* dst2, const RowGeom& rg,
                    const Cx<T>* tw, const Forcing& F) {
  constexpr int pb0 = row_pb<T, L>(0);
  constexpr int pbs = std::max(1, pb0 / 4);
  const bool few = (nrows + 2 * pb0 - 1) / (2 * pb0) < g_cus;
  auto go = [&](auto pbc) {
    constexpr int PB = decltype(pbc)::value;
    constexpr int NT = PB * fast::FftShape<L>::LP;
    dim3 grid((nrows + 2 * PB - 1) / (2 * PB));
    if (mode == ROW_PHYS)
      hipLaunchKernelGGL((fast::row_fast_per<T, L, PB, ROW_PHYS>), grid, dim3(NT), 0, s, src, dst, dst2, rg, tw, F);
    else if (mode == ROW_FWD_USER)
      hipLaunchKernelGGL((fast::row_fast_per<T, L, PB, ROW_FWD_USER>), grid, dim3(NT), 0, s, src, dst, dst2, rg, tw, F);
    else
      hipLaunchKernelGGL((fast::row_fast_per<T, L, PB, ROW_INV_USER>), grid, dim3(NT), 0, s, src, dst, dst2, rg, tw, F);
  };
  if (few)
    go(std::integral_constant<int, pbs>());
  else
    go(std::integral_constant<int, pb0>());
}

template <typename T>
bool try_row_fast_per(const eife_grid_s* g, int mode, int count, hipStream_t s, const T* src, T* dst, T* dst2,
                      const RowGeom& rg, const Cx<T>* tw, const Forcing& F, const RowInst<T>* ri) {
  if (g->transform != EIFE_TX_FFT || ri || count != 1 || !per_fast_len(g->N[0])) return false;
  if (mode != ROW_PHYS && mode != ROW_FWD_USER && mode != ROW_INV_USER) return false;
  switch (g->N[0]) {
    case 128: row_per_launch<T, 128>(mode, rg.nrows, s, src, dst, dst2, rg, tw, F); return true;
    case 256: row_per_launch<T, 256>(mode, rg.nrows, s, src, dst, dst2, rg, tw, F); return true;
    case 512: row_per_launch<T, 512>(mode, rg.nrows, s, src, dst, dst2, rg, tw, F); return true;
  }
  return false;
}

template <typename T, int L>
void col_per_launch(int mode, int pitch, int outer, hipStream_t s, T* W, T* H, const ColGeom& cg, const Cx<T>* tw,
                    const Diag& dg) {
  constexpr int pb0 = col_pb<T, L>(0);
  constexpr int pbs = std::max(1, pb0 / 8);
  const bool few = (pitch / (2 * pb0)) * outer < g_cus;
  auto go = [&](auto pbc) {
    constexpr int PB = decltype(pbc)::value;
    constexpr int PPW = col_ppw<T, L, PB>();
    constexpr int NT = PB / PPW * fast::FftShape<L>::LP;
    dim3 grid(pitch / (2 * PB), outer);
    if (mode == COL_PLAIN)
      hipLaunchKernelGGL((fast::col_fast_per<T, L, PB, PPW, COL_PLAIN>), grid, dim3(NT), 0, s, W, H, cg, tw, dg);
    else if (mode == COL_PLAIN_INV)
      hipLaunchKernelGGL((fast::col_fast_per<T, L, PB, PPW, COL_PLAIN_INV>), grid, dim3(NT), 0, s, W, H, cg, tw, dg);
    else if (mode == COL_STAGE_A)
      hipLaunchKernelGGL((fast::col_fast_per<T, L, PB, PPW, COL_STAGE_A>), grid, dim3(NT), 0, s, W, H, cg, tw, dg);
    else if (mode == COL_STAGE_B)
      hipLaunchKernelGGL((fast::col_fast_per<T, L, PB, PPW, COL_STAGE_B>), grid, dim3(NT), 0, s, W, H, cg, tw, dg);
    else
      hipLaunchKernelGGL((fast::col_fast_per<T, L, PB, PPW, COL_ETD1>), grid, dim3(NT), 0, s, W, H, cg, tw, dg);
  };
  if (few)
    go(std::integral_constant<int, pbs>());
  else
    go(std::integral_constant<int, pb0>());
}

template <typename T>
bool try_col_fast_per(const eife_grid_s* g, int axis, int mode, int outer, int count, hipStream_t s, T* W, T* H,
                      const ColGeom& cg, const Cx<T>* tw, const Diag& dg, const ColInst<T>* ci) {
  if (g->transform != EIFE_TX_FFT || ci || count != 1 || !per_fast_len(g->N[axis]) || mode >= COL_S3_1) return false;
  switch (g->N[axis]) {
    case 128: col_per_launch<T, 128>(mode, g->pitch, outer, s, W, H, cg, tw, dg); return true;
    case 256: col_per_launch<T, 256>(mode, g->pitch, outer, s, W, H, cg, tw, dg); return true;
    case 512: col_per_launch<T, 512>(mode, g->pitch, outer, s, W, H, cg, tw, dg); return true;
  }
  return false;
}

// Lines of 1024, 2048 and 4096 intervals (2048-, 4096- and 8192-point odd
// extensions): one line pair per block (eife_long.hpp); single grids,
// non-periodic.
inline bool long_len(int N) { return N == 1024 || N == 2048 || N == 4096; }

template <typename T, int L>
void row_long_launch(int mode, int nrows, hipStream_t s, const T* src, T* dst, T* dst2, const RowGeom& rg,
                     const Cx<T>* tw, const Forcing& F) {
  constexpr int NT = lng::Shape<L>::NT;
  const dim3 grid((nrows + 1) / 2);
  if (!launch_shape_ok(grid, NT, lng::Shape<L>::BUF * sizeof(Cx<T>))) return;
  if (mode == ROW_PHYS) {
    if (F.kind == FK_AC)
      hipLaunchKernelGGL((lng::row_long<T, L, ROW_PHYS, fast::RK_AC>), grid, dim3(NT), 0, s, src, dst, dst2, rg, tw, F);
    else
      hipLaunchKernelGGL((lng::row_long<T, L, ROW_PHYS, fast::RK_GENERIC>), grid, dim3(NT), 0, s, src, dst, dst2, rg, tw,
                         F);
  } else if (mode == ROW_FWD_USER) {
    hipLaunchKernelGGL((lng::row_long<T, L, ROW_FWD_USER, fast::RK_GENERIC>), grid, dim3(NT), 0, s, src, dst, dst2, rg,
                       tw, F);
  } else {
    hipLaunchKernelGGL((lng::row_long<T, L, ROW_INV_USER, fast::RK_GENERIC>), grid, dim3(NT), 0, s, src, dst, dst2, rg,
                       tw, F);
  }
}

template <typename T, int L>
void col_long_launch(int mode, int pitch, int outer, hipStream_t s, T* W, T* H, const ColGeom& cg, const Cx<T>* tw,
                     const Diag& dg) {
  constexpr int NT = lng::Shape<L>::NT;
  if constexpr (2 * lng::Shape<L>::BUF * sizeof(Cx<T>) <= 160 * 1024) {
    // two column pairs (a 16- or 32-byte row piece) per block of 2 NT threads (FP32, and FP64 up to
    // 4096 points); the pitch is a multiple of 32
    const dim3 grid(pitch / 4, outer);
    if (!launch_shape_ok(grid, 2 * NT, 2 * lng::Shape<L>::BUF * sizeof(Cx<T>))) return;
    if (mode == COL_PLAIN)
      hipLaunchKernelGGL((lng::col_long4<T, L, COL_PLAIN>), grid, dim3(2 * NT), 0, s, W, H, cg, tw, dg);
    else if (mode == COL_STAGE_A)
      hipLaunchKernelGGL((lng::col_long4<T, L, COL_STAGE_A>), grid, dim3(2 * NT), 0, s, W, H, cg, tw, dg);
    else if (mode == COL_STAGE_B)
      hipLaunchKernelGGL((lng::col_long4<T, L, COL_STAGE_B>), grid, dim3(2 * NT), 0, s, W, H, cg, tw, dg);
    else
      hipLaunchKernelGGL((lng::col_long4<T, L, COL_ETD1>), grid, dim3(2 * NT), 0, s, W, H, cg, tw, dg);
  } else {
    const dim3 grid(pitch / 2, outer);
    if (!launch_shape_ok(grid, NT, lng::Shape<L>::BUF * sizeof(Cx<T>))) return;
    if (mode == COL_PLAIN)
      hipLaunchKernelGGL((lng::col_long<T, L, COL_PLAIN>), grid, dim3(NT), 0, s, W, H, cg, tw, dg);
    else if (mode == COL_STAGE_A)
      hipLaunchKernelGGL((lng::col_long<T, L, COL_STAGE_A>), grid, dim3(NT), 0, s, W, H, cg, tw, dg);
    else if (mode == COL_STAGE_B)
      hipLaunchKernelGGL((lng::col_long<T, L, COL_STAGE_B>), grid, dim3(NT), 0, s, W, H, cg, tw, dg);
    else
      hipLaunchKernelGGL((lng::col_long<T, L, COL_ETD1>), grid, dim3(NT), 0, s, W, H, cg, tw, dg);
  }
}

template <typename T>
bool try_row_fast(const eife_grid_s* g, int var, int mode, int count, hipStream_t s, const T* src, T* dst, T* dst2,
                  const RowGeom& rg, const Cx<T>* tw, const Forcing& F, const RowInst<T>* ri) {
  if (g->per[0]) return try_row_fast_per<T>(g, mode, count, s, src, dst, dst2, rg, tw, F, ri);
  // the traveling wave's boundary code runs in the generic row pass only
  if (g->transform != EIFE_TX_FFT || F.kind == FK_EX52) return false;
  if (long_len(g->N[0])) {
    if (count != 1 || ri || (mode != ROW_PHYS && mode != ROW_FWD_USER && mode != ROW_INV_USER)) return false;
    if (g->N[0] == 1024)
      row_long_launch<T, 2048>(mode, rg.nrows, s, src, dst, dst2, rg, tw, F);
    else if (g->N[0] == 2048)
      row_long_launch<T, 4096>(mode, rg.nrows, s, src, dst, dst2, rg, tw, F);
    else
      row_long_launch<T, 8192>(mode, rg.nrows, s, src, dst, dst2, rg, tw, F);
    return true;
  }
  if (!fast_len<T>(g->N[0])) return false;
  switch (g->N[0]) {
    case 64: row_fast_launch<T, 128>(var, mode, rg.nrows, count, s, src, dst, dst2, rg, tw, F, ri); return true;
    case 128: row_fast_launch<T, 256>(var, mode, rg.nrows, count, s, src, dst, dst2, rg, tw, F, ri); return true;
    case 256: row_fast_launch<T, 512>(var, mode, rg.nrows, count, s, src, dst, dst2, rg, tw, F, ri); return true;
    case 512: row_fast_launch<T, 1024>(var, mode, rg.nrows, count, s, src, dst, dst2, rg, tw, F, ri); return true;
    case 192: row_fast_launch<T, 384>(var, mode, rg.nrows, count, s, src, dst, dst2, rg, tw, F, ri); return true;
    case 384:
      if constexpr (sizeof(T) == 4) {
        row_fast_launch<T, 768>(var, mode, rg.nrows, count, s, src, dst, dst2, rg, tw, F, ri);
        return true;
      }
      return false;
  }
  return false;
}

template <typename T>
bool try_col_fast(const eife_grid_s* g, int var, int axis, int mode, int outer, int count, hipStream_t s, T* W, T* H,
                  const ColGeom& cg, const Cx<T>* tw, const Diag& dg, const ColInst<T>* ci) {
  if (g->per[axis]) return try_col_fast_per<T>(g, axis, mode, outer, count, s, W, H, cg, tw, dg, ci);
  if (g->transform != EIFE_TX_FFT) return false;
  if (long_len(g->N[axis])) {
    if (count != 1 || ci || mode > COL_ETD1) return false;
    if (g->N[axis] == 1024)
      col_long_launch<T, 2048>(mode, g->pitch, outer, s, W, H, cg, tw, dg);
    else if (g->N[axis] == 2048)
      col_long_launch<T, 4096>(mode, g->pitch, outer, s, W, H, cg, tw, dg);
    else
      col_long_launch<T, 8192>(mode, g->pitch, outer, s, W, H, cg, tw, dg);
    return true;
  }
  if (!fast_len<T>(g->N[axis])) return false;
  switch (g->N[axis]) {
    case 64: col_fast_launch<T, 128>(var, mode, g->pitch, outer, count, s, W, H, cg, tw, dg, ci); return true;
    case 128: col_fast_launch<T, 256>(var, mode, g->pitch, outer, count, s, W, H, cg, tw, dg, ci); return true;
    case 256: col_fast_launch<T, 512>(var, mode, g->pitch, outer, count, s, W, H, cg, tw, dg, ci); return true;
    case 512: col_fast_launch<T, 1024>(var, mode, g->pitch, outer, count, s, W, H, cg, tw, dg, ci); return true;
    case 192: col_fast_launch<T, 384>(var, mode, g->pitch, outer, count, s, W, H, cg, tw, dg, ci); return true;
    case 384:
      if constexpr (sizeof(T) == 4) {
        col_fast_launch<T, 768>(var, mode, g->pitch, outer, count, s, W, H, cg, tw, dg, ci);
        return true;
      }
      return false;
  }
  return false;
}

template <typename T, bool BATR, int NT = kThreads>
void row_generic_go(int mode, dim3 grid, size_t shm, hipStream_t s, const T* src, T* dst, T* dst2, const RowGeom& rg,
                    const Cx<T>* tw, const Forcing& F, const RowInst<T>* ri) {
  if (mode == ROW_PHYS)
    hipLaunchKernelGGL((row_pass<T, ROW_PHYS, BATR, NT>), grid, dim3(NT), shm, s, src, dst, dst2, rg, tw, F, ri);
  else if (mode == ROW_FWD_USER)
    hipLaunchKernelGGL((row_pass<T, ROW_FWD_USER, BATR, NT>), grid, dim3(NT), shm, s, src, dst, dst2, rg, tw, F, ri);
  else
    hipLaunchKernelGGL((row_pass<T, ROW_INV_USER, BATR, NT>), grid, dim3(NT), shm, s, src, dst, dst2, rg, tw, F, ri);
}

template <typename T, bool BATC, int NT = kThreads>
void col_generic_go(int mode, dim3 grid, size_t shm, hipStream_t s, T* W, T* H, const ColGeom& cg, const Cx<T>* tw,
                    const Diag& dg, const ColInst<T>* ci) {
  if constexpr (!BATC) {
    if (mode == COL_S3_1) {
      hipLaunchKernelGGL((col_pass<T, COL_S3_1, false, NT>), grid, dim3(NT), shm, s, W, H, cg, tw, dg, ci);
      return;
    }
    if (mode == COL_S3_2) {
      hipLaunchKernelGGL((col_pass<T, COL_S3_2, false, NT>), grid, dim3(NT), shm, s, W, H, cg, tw, dg, ci);
      return;
    }
    if (mode == COL_S3_3) {
      hipLaunchKernelGGL((col_pass<T, COL_S3_3, false, NT>), grid, dim3(NT), shm, s, W, H, cg, tw, dg, ci);
      return;
    }
  }
  if (mode == COL_PLAIN)
    hipLaunchKernelGGL((col_pass<T, COL_PLAIN, BATC, NT>), grid, dim3(NT), shm, s, W, H, cg, tw, dg, ci);
  else if (mode == COL_STAGE_A)
    hipLaunchKernelGGL((col_pass<T, COL_STAGE_A, BATC, NT>), grid, dim3(NT), shm, s, W, H, cg, tw, dg, ci);
  else if (mode == COL_STAGE_B)
    hipLaunchKernelGGL((col_pass<T, COL_STAGE_B, BATC, NT>), grid, dim3(NT), shm, s, W, H, cg, tw, dg, ci);
  else
    hipLaunchKernelGGL((col_pass<T, COL_ETD1, BATC, NT>), grid, dim3(NT), shm, s, W, H, cg, tw, dg, ci);
}

// Periodic lines (generic passes only).
template <typename T, int NT = kThreads>
void row_periodic_go(int mode, dim3 grid, size_t shm, hipStream_t s, const T* src, T* dst, T* dst2,
                     const RowGeom& rg, const Cx<T>* tw, const Forcing& F) {
  if (mode == ROW_PHYS)
    hipLaunchKernelGGL((row_pass_per<T, ROW_PHYS, NT>), grid, dim3(NT), shm, s, src, dst, dst2, rg, tw, F);
  else if (mode == ROW_FWD_USER)
    hipLaunchKernelGGL((row_pass_per<T, ROW_FWD_USER, NT>), grid, dim3(NT), shm, s, src, dst, dst2, rg, tw, F);
  else
    hipLaunchKernelGGL((row_pass_per<T, ROW_INV_USER, NT>), grid, dim3(NT), shm, s, src, dst, dst2, rg, tw, F);
}

template <typename T, int NT = kThreads>
void col_periodic_go(int mode, dim3 grid, size_t shm, hipStream_t s, T* W, T* H, const ColGeom& cg,
                     const Cx<T>* tw, const Diag& dg) {
  if (mode == COL_PLAIN)
    hipLaunchKernelGGL((col_pass_per<T, COL_PLAIN, NT>), grid, dim3(NT), shm, s, W, H, cg, tw, dg);
  else if (mode == COL_PLAIN_INV)
    hipLaunchKernelGGL((col_pass_per<T, COL_PLAIN_INV, NT>), grid, dim3(NT), shm, s, W, H, cg, tw, dg);
  else if (mode == COL_STAGE_A)
    hipLaunchKernelGGL((col_pass_per<T, COL_STAGE_A, NT>), grid, dim3(NT), shm, s, W, H, cg, tw, dg);
  else if (mode == COL_STAGE_B)
    hipLaunchKernelGGL((col_pass_per<T, COL_STAGE_B, NT>), grid, dim3(NT), shm, s, W, H, cg, tw, dg);
  else if (mode == COL_S3_1)
    hipLaunchKernelGGL((col_pass_per<T, COL_S3_1, NT>), grid, dim3(NT), shm, s, W, H, cg, tw, dg);
  else if (mode == COL_S3_2)
    hipLaunchKernelGGL((col_pass_per<T, COL_S3_2, NT>), grid, dim3(NT), shm, s, W, H, cg, tw, dg);
  else if (mode == COL_S3_3)
    hipLaunchKernelGGL((col_pass_per<T, COL_S3_3, NT>), grid, dim3(NT), shm, s, W, H, cg, tw, dg);
  else
    hipLaunchKernelGGL((col_pass_per<T, COL_ETD1, NT>), grid, dim3(NT), shm, s, W, H, cg, tw, dg);
}

// ---------------------------------------------------------------------------
// Split-BF16 matrix-core transform (single grids, FP32).

int gemm_kp(int n) {
  int kp = 64;
  while (kp < n) kp *= 2;
  return kp;
}

uint16_t bf16_bits(float x) {  // round to nearest even
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

float bf16_value(uint16_t b) {
  const uint32_t u = uint32_t(b) << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}

// S_mk = sqrt(2/N) sin((m+1)(k+1) pi / N) for m, k < N-1, zero padded to kp x kp,
// split into hi = bf16(s) and lo = bf16(s - hi).
int build_smat(eife_grid_s* g, int a) {
  const int n = g->n[a], N = g->N[a], kp = gemm_kp(n);
  std::vector<uint16_t> v(size_t(2) * kp * kp, 0);
  const double sc = std::sqrt(2.0 / N);
  for (int m = 0; m < n; ++m)
    for (int k = 0; k < n; ++k) {
      const long long j = (long long)(m + 1) * (k + 1) % (2 * N);  // sin is 2N-periodic in j
      const double sv = sc * std::sin(M_PI * double(j) / N);
      const uint16_t hi = bf16_bits(float(sv));
      v[size_t(m) * kp + k] = hi;
      v[size_t(kp) * kp + size_t(m) * kp + k] = bf16_bits(float(sv - double(bf16_value(hi))));
    }
  hipFree(g->smat[a]);
  g->smat[a] = nullptr;
  if (hipMalloc(&g->smat[a], v.size() * 2) != hipSuccess) return fail(EIFE_ENOMEM, "sine matrix allocation failed");
  HIP_TRY(hipMemcpy(g->smat[a], v.data(), v.size() * 2, hipMemcpyHostToDevice));
  g->kp[a] = kp;
  return EIFE_OK;
}

gemm::SMat smat_of(const eife_grid_s* g, int a) {
  const __bf16* p = static_cast<const __bf16*>(g->smat[a]);
  return gemm::SMat{p, p + size_t(g->kp[a]) * g->kp[a]};
}

template <int KP>
int gemm_attrs() {
  const int shm = int(gemm::Shape<KP>::LDS);
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm::gemm_row<KP, ROW_PHYS, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm::gemm_row<KP, ROW_PHYS, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm::gemm_row<KP, ROW_FWD_USER, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm::gemm_row<KP, ROW_INV_USER, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm::gemm_col<KP, COL_PLAIN>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm::gemm_col<KP, COL_STAGE_A>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm::gemm_col<KP, COL_STAGE_B>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm::gemm_col<KP, COL_ETD1>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  return EIFE_OK;
}

int gemm_attrs_all() {
  static int done = 0;  // per process; the attribute holds for every device
  if (done) return EIFE_OK;
  int r = gemm_attrs<64>();
  if (r == EIFE_OK) r = gemm_attrs<128>();
  if (r == EIFE_OK) r = gemm_attrs<256>();
  if (r == EIFE_OK) r = gemm_attrs<512>();
  if (r == EIFE_OK) r = gemm_attrs<1024>();
  if (r == EIFE_OK) done = 1;
  return r;
}

template <int KP>
void gemm_row_go(int mode, bool ac, hipStream_t s, const float* src, float* dst, float* dst2, const RowGeom& rg,
                 gemm::SMat S, const Forcing& F) {
  using Sh = gemm::Shape<KP>;
  const dim3 grid((rg.nrows + Sh::TL - 1) / Sh::TL);
  const dim3 blk(Sh::THREADS);
  if (mode == ROW_PHYS && ac)
    hipLaunchKernelGGL((gemm::gemm_row<KP, ROW_PHYS, true>), grid, blk, Sh::LDS, s, src, dst, dst2, rg, S, F);
  else if (mode == ROW_PHYS)
    hipLaunchKernelGGL((gemm::gemm_row<KP, ROW_PHYS, false>), grid, blk, Sh::LDS, s, src, dst, dst2, rg, S, F);
  else if (mode == ROW_FWD_USER)
    hipLaunchKernelGGL((gemm::gemm_row<KP, ROW_FWD_USER, false>), grid, blk, Sh::LDS, s, src, dst, dst2, rg, S, F);
  else
    hipLaunchKernelGGL((gemm::gemm_row<KP, ROW_INV_USER, false>), grid, blk, Sh::LDS, s, src, dst, dst2, rg, S, F);
}

template <int KP>
void gemm_col_go(int mode, int pitch, int outer, hipStream_t s, float* W, float* H, const ColGeom& cg,
                 gemm::SMat S, const Diag& dg) {
  using Sh = gemm::Shape<KP>;
  const dim3 grid((pitch + Sh::TL - 1) / Sh::TL, outer);
  const dim3 blk(Sh::THREADS);
  if (mode == COL_PLAIN)
    hipLaunchKernelGGL((gemm::gemm_col<KP, COL_PLAIN>), grid, blk, Sh::LDS, s, W, H, cg, pitch, S, dg);
  else if (mode == COL_STAGE_A)
    hipLaunchKernelGGL((gemm::gemm_col<KP, COL_STAGE_A>), grid, blk, Sh::LDS, s, W, H, cg, pitch, S, dg);
  else if (mode == COL_STAGE_B)
    hipLaunchKernelGGL((gemm::gemm_col<KP, COL_STAGE_B>), grid, blk, Sh::LDS, s, W, H, cg, pitch, S, dg);
  else
    hipLaunchKernelGGL((gemm::gemm_col<KP, COL_ETD1>), grid, blk, Sh::LDS, s, W, H, cg, pitch, S, dg);
}

template <typename T>
bool try_row_gemm(const eife_grid_s* g, int mode, hipStream_t s, const T* src, T* dst, T* dst2, const RowGeom& rg,
                  const Forcing& F) {
  if constexpr (sizeof(T) != 4) {
    return false;
  } else {
    // the traveling wave's boundary code runs in the generic row pass only
    if (g->transform != EIFE_TX_GEMM_SPLITBF16 || F.kind == FK_EX52) return false;
    const gemm::SMat S = smat_of(g, 0);
    const bool ac = F.kind == FK_AC;
    switch (g->kp[0]) {
      case 64: gemm_row_go<64>(mode, ac, s, src, dst, dst2, rg, S, F); return true;
      case 128: gemm_row_go<128>(mode, ac, s, src, dst, dst2, rg, S, F); return true;
      case 256: gemm_row_go<256>(mode, ac, s, src, dst, dst2, rg, S, F); return true;
      case 512: gemm_row_go<512>(mode, ac, s, src, dst, dst2, rg, S, F); return true;
      case 1024: gemm_row_go<1024>(mode, ac, s, src, dst, dst2, rg, S, F); return true;
    }
    return false;
  }
}

template <typename T>
bool try_col_gemm(const eife_grid_s* g, int axis, int mode, int outer, hipStream_t s, T* W, T* H, const ColGeom& cg,
                  const Diag& dg) {
  if constexpr (sizeof(T) != 4) {
    return false;
  } else {
    if (g->transform != EIFE_TX_GEMM_SPLITBF16) return false;
    const gemm::SMat S = smat_of(g, axis);
    switch (g->kp[axis]) {
      case 64: gemm_col_go<64>(mode, g->pitch, outer, s, W, H, cg, S, dg); return true;
      case 128: gemm_col_go<128>(mode, g->pitch, outer, s, W, H, cg, S, dg); return true;
      case 256: gemm_col_go<256>(mode, g->pitch, outer, s, W, H, cg, S, dg); return true;
      case 512: gemm_col_go<512>(mode, g->pitch, outer, s, W, H, cg, S, dg); return true;
      case 1024: gemm_col_go<1024>(mode, g->pitch, outer, s, W, H, cg, S, dg); return true;
    }
    return false;
  }
}

// The first reaction of a run is fused into the forward row pass of the
// prologue (ROW_FWD_PHYS) wherever the specialised row kernels run.
template <typename T>
bool fused_first_row(const eife_grid_s* g, int f_kind) {
  return g->transform == EIFE_TX_FFT && !g->per[0] && fast_len<T>(g->N[0]) && f_kind != EIFE_F_TRAVELING_WAVE;
}

// The last row pass of a step can also sum (u - u_n)^2 per line pair
// (ROW_INV_CHG) on 2D grids whose rows run on the specialised kernels with one
// wavefront per line pair (N_x = 256 or 512).
template <typename T>
bool change_epilogue(const eife_grid_s* g) {
  return g->d == 2 && g->transform == EIFE_TX_FFT && !g->per[0] && (g->N[0] == 256 || g->N[0] == 512);
}

// A launch of one pass over `count` instances shaped like grid `g`.
struct Batchlet {
  int count = 1;
  const void* rinst = nullptr;  // RowInst<T>[count] (device) or null
  const void* cinst = nullptr;  // ColInst<T>[count] (device) or null
  int var_row = 0, var_col = 0;  // tuned launch variants
  int prow = 0, pcol = 0;        // generic-kernel pairs per block (0 = the grid's default)
};

template <typename T>
int launch_row(eife_grid_s* g, int mode, const T* src, int64_t ld_src, T* dst, int64_t ld_dst, T* dst2,
               const Forcing& F, hipStream_t s, const Batchlet& B = Batchlet(), double* chg = nullptr) {
  if (mode == ROW_INV_CHG && (!chg || !change_epilogue<T>(g)))
    return fail(EIFE_EUNSUPPORTED, "row pass with change sums on this grid");
  RowGeom rg;
  rg.chg = chg;
  rg.n = g->n[0];
  rg.nrows = g->nlines_total();
  rg.ny = g->n[1];
  rg.ld_src = ld_src;
  rg.ld_dst = ld_dst;
  rg.pl = g->plan[0];
  rg.P = B.prow > 0 ? B.prow : g->prow;
  rg.ls = rg.pl.L + 1;
  const RowInst<T>* ri = static_cast<const RowInst<T>*>(B.rinst);
  const Cx<T>* tw = reinterpret_cast<const Cx<T>*>(g->tw[0]);
  const int pidx = prof_begin(g, mode == ROW_PHYS ? EIFE_PASS_ROW_PHYS
                                 : (mode == ROW_FWD_USER || mode == ROW_FWD_PHYS) ? EIFE_PASS_ROW_FWD
                                                                                   : EIFE_PASS_ROW_INV, s);
  if (mode == ROW_FWD_PHYS && !fused_first_row<T>(g, F.kind)) return fail(EIFE_EUNSUPPORTED, "fused first row pass");
  g_bad_launch = nullptr;
  if (!(B.count == 1 && !ri && try_row_gemm<T>(g, mode, s, src, dst, dst2, rg, F)) &&
      !try_row_fast<T>(g, B.var_row, mode, B.count, s, src, dst, dst2, rg, tw, F, ri)) {
    const size_t shm = lds_bytes(g, rg.P, rg.pl.L);
    dim3 grid((rg.nrows + 2 * rg.P - 1) / (2 * rg.P), B.count);
    if (g->per[0]) {
      if (ri || mode == ROW_FWD_PHYS) return fail(EIFE_EUNSUPPORTED, "periodic row pass variant");
      if (long_lines<T>(rg.pl.L))
        row_periodic_go<T, kLongThreads>(mode, grid, shm, s, src, dst, dst2, rg, tw, F);
      else
        row_periodic_go<T>(mode, grid, shm, s, src, dst, dst2, rg, tw, F);
    } else if (ri)
      row_generic_go<T, true>(mode, grid, shm, s, src, dst, dst2, rg, tw, F, ri);
    else
      if (long_lines<T>(rg.pl.L))
        row_generic_go<T, false, kLongThreads>(mode, grid, shm, s, src, dst, dst2, rg, tw, F, ri);
      else
        row_generic_go<T, false>(mode, grid, shm, s, src, dst, dst2, rg, tw, F, ri);
  }
  if (g_bad_launch) return fail(EIFE_EINVAL, "%s", g_bad_launch);
  HIP_TRY(hipGetLastError());
  prof_end(g, pidx, s);
  return EIFE_OK;
}

// axis = 1 (y) or 2 (z)
template <typename T>
int launch_col(eife_grid_s* g, int axis, int mode, T* W, T* H, const Diag& dg, hipStream_t s,
               const Batchlet& B = Batchlet()) {
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
  cg.ncols = g->n[0];
  cg.pl = g->plan[axis];
  cg.P = B.pcol > 0 ? B.pcol : g->pcol[axis];
  while (g->pitch % (2 * cg.P) != 0) cg.P--;
  cg.ls = cg.pl.L + 1;
  const ColInst<T>* ci = static_cast<const ColInst<T>*>(B.cinst);
  const Cx<T>* tw = reinterpret_cast<const Cx<T>*>(g->tw[axis]);
  int kind = EIFE_PASS_MID;
  if (!(axis == 1 && g->d == 3)) {
    kind = mode == COL_PLAIN ? EIFE_PASS_LAST_PLAIN
           : (mode == COL_STAGE_A || mode == COL_S3_1) ? EIFE_PASS_LAST_A
           : (mode == COL_STAGE_B || mode == COL_S3_2 || mode == COL_S3_3) ? EIFE_PASS_LAST_B : EIFE_PASS_LAST_ETD1;
  }
  const int pidx = prof_begin(g, kind, s);
  // the three-stage column passes: specialised (one tile per block) or generic kernels, no matrix-core variant
  const bool s3 = mode >= COL_S3_1;
  g_bad_launch = nullptr;
  if ((s3 || !(B.count == 1 && !ci && try_col_gemm<T>(g, axis, mode, outer, s, W, H, cg, dg))) &&
      !try_col_fast<T>(g, B.var_col, axis, mode, outer, B.count, s, W, H, cg, tw, dg, ci)) {
    const size_t shm = lds_bytes(g, cg.P, cg.pl.L);
    dim3 grid(g->pitch / (2 * cg.P), outer, B.count);
    if (g->per[axis]) {
      if (ci) return fail(EIFE_EUNSUPPORTED, "periodic batched column pass");
      if (long_lines<T>(cg.pl.L))
        col_periodic_go<T, kLongThreads>(mode, grid, shm, s, W, H, cg, tw, dg);
      else
        col_periodic_go<T>(mode, grid, shm, s, W, H, cg, tw, dg);
    } else if (ci)
      col_generic_go<T, true>(mode, grid, shm, s, W, H, cg, tw, dg, ci);
    else
      if (long_lines<T>(cg.pl.L))
        col_generic_go<T, false, kLongThreads>(mode, grid, shm, s, W, H, cg, tw, dg, ci);
      else
        col_generic_go<T, false>(mode, grid, shm, s, W, H, cg, tw, dg, ci);
  }
  if (g_bad_launch) return fail(EIFE_EINVAL, "%s", g_bad_launch);
  HIP_TRY(hipGetLastError());
  prof_end(g, pidx, s);
  return EIFE_OK;
}

#define RET_IF(x)             \
  do {                        \
    int _r = (x);             \
    if (_r != EIFE_OK) return _r; \
  } while (0)

// Steps per chunk of a variable-step run: the chunk's tables take at most
// 16 MB (at least one step).
constexpr int64_t kVarChunkMax = 512;
constexpr int64_t kVarChunkBytes = int64_t(16) << 20;

int ensure_step_tables(eife_grid_s* g) {
  if (g->vchunk) return EIFE_OK;
  const int64_t stride = step_table_stride(g);
  const int64_t chunk = std::max<int64_t>(1, std::min(kVarChunkMax, kVarChunkBytes / (stride * 8)));
  const size_t bytes = 2 * size_t(chunk * stride) * sizeof(double);
  if (hipMalloc(reinterpret_cast<void**>(&g->vtab), bytes) != hipSuccess) {
    g->vtab = nullptr;
    return fail(EIFE_ENOMEM, "variable-step table allocation failed");
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&g->vhost), bytes, hipHostMallocDefault) != hipSuccess) {
    hipFree(g->vtab);
    g->vtab = nullptr;
    g->vhost = nullptr;
    return fail(EIFE_ENOMEM, "variable-step staging allocation failed");
  }
  for (int b = 0; b < 2; ++b) {
    if (hipEventCreateWithFlags(&g->vev[b], hipEventDisableTiming) != hipSuccess) {
      for (int c = 0; c < b; ++c) hipEventDestroy(g->vev[c]);
      g->vev[0] = g->vev[1] = nullptr;
      hipFree(g->vtab);
      hipHostFree(g->vhost);
      g->vtab = nullptr;
      g->vhost = nullptr;
      return fail(EIFE_EHIP, "cannot create the variable-step events");
    }
  }
  g->vchunk = chunk;
  return EIFE_OK;
}

// taus (host, n_steps entries) selects variable steps: t_{n+1} = t_n + tau_n
// (running sum in double), every factor formed with tau_n; null: uniform
// steps of the grid's tau, t_n = t0 + n tau.
template <typename T>
int run_steps(eife_grid_s* g, const T* u, int64_t n_steps, int f_kind, double t0, hipStream_t s,
              const double* taus = nullptr, T* u_out = nullptr, double* chg = nullptr) {
  T* W = static_cast<T*>(g->W);
  T* H = static_cast<T*>(g->H);
  const Diag dg_fixed = make_diag(g);
  const Diag& dg0 = dg_fixed;
  const bool three = g->d == 3;
  const int last = three ? 2 : 1;
  // the y pass after the last-axis pass goes back to nodal y (the sine
  // transform is its own inverse, the real Fourier transform is not)
  const int inv_plain = g->per[1] ? COL_PLAIN_INV : COL_PLAIN;
  const Forcing F0 = make_forcing(g, f_kind, t0);
  // prologue: H = S u and W = S_x u, or W = S_x f(t0, u) when the first
  // reaction is fused in
  const bool fused = n_steps > 0 && fused_first_row<T>(g, f_kind);
  RET_IF(launch_row<T>(g, fused ? ROW_FWD_PHYS : ROW_FWD_USER, u, g->n[0], W, g->pitch, H, F0, s));
  if (three) RET_IF(launch_col<T>(g, 1, COL_PLAIN, H, H, dg0, s));
  RET_IF(launch_col<T>(g, last, COL_PLAIN, H, H, dg0, s));
  const int64_t stride = taus ? step_table_stride(g) : 0;
  double tv = t0;  // running time of a variable-step run
  for (int64_t st = 0; st < n_steps; ++st) {
    double tau = g->tau;
    Diag dg_var;
    if (taus) {
      const int64_t j = st % g->vchunk;
      const int64_t c = st / g->vchunk;
      double* dev = g->vtab + (c & 1) * g->vchunk * stride;
      if (j == 0) {
        // chunk c goes to buffer c & 1 while the device may still run chunk
        // c - 1 from the other one.  The staging half is rewritten once the
        // last copy out of it (chunk c - 2, or a previous call's) has
        // completed (its event; an event never recorded does not wait); the
        // device half is rewritten in stream order, after the kernels that
        // read it (calls on one grid are ordered by the caller, as for W, H).
        double* host = g->vhost + (c & 1) * g->vchunk * stride;
        HIP_TRY(hipEventSynchronize(g->vev[c & 1]));
        const int64_t cnt = std::min(g->vchunk, n_steps - st);
        for (int64_t q = 0; q < cnt; ++q) {
          double* blk = host + q * stride;
          for (int ax = 0; ax < 3; ++ax) {
            fill_phi(g, ax, taus[st + q], blk);
            blk += kStepArrays * g->tablen[ax];
          }
        }
        HIP_TRY(hipMemcpyAsync(dev, host, size_t(cnt * stride) * sizeof(double), hipMemcpyHostToDevice, s));
        HIP_TRY(hipEventRecord(g->vev[c & 1], s));
      }
      tau = taus[st];
      if (st > 0) tv += taus[st - 1];
      dg_var = make_diag_at(g, dev + j * stride, tau);
    }
    const Diag& dg = taus ? dg_var : dg_fixed;
    const double tn = taus ? tv : t0 + double(st) * g->tau;
    // stage i: reaction at t_n + c_i tau, transforms, the stage's diagonal update
    static const int kModes[4][3] = {{0, 0, 0}, {COL_ETD1, 0, 0}, {COL_STAGE_A, COL_STAGE_B, 0},
                                     {COL_S3_1, COL_S3_2, COL_S3_3}};
    const double nodes[3] = {0.0, node_c2(g), g->c3_3};
    for (int i = 0; i < g->stages; ++i) {
      if (!(fused && st == 0 && i == 0))
        RET_IF(launch_row<T>(g, ROW_PHYS, W, g->pitch, W, g->pitch, nullptr,
                             make_forcing(g, f_kind, i ? tn + nodes[i] * tau : tn), s));
      if (three) RET_IF(launch_col<T>(g, 1, COL_PLAIN, W, H, dg, s));
      RET_IF(launch_col<T>(g, last, kModes[g->stages][i], W, H, dg, s));
      if (three) RET_IF(launch_col<T>(g, 1, inv_plain, W, H, dg, s));
    }
  }
  // epilogue: u = S_x^{-1} W (u_out: only the prologue reads u)
  if (chg)  // u is read again here: the sums of (u_out - u)^2 per line pair
    RET_IF(launch_row<T>(g, ROW_INV_CHG, W, g->pitch, u_out, g->n[0], const_cast<T*>(u), F0, s, Batchlet(), chg));
  else
    RET_IF(launch_row<T>(g, ROW_INV_USER, W, g->pitch, u_out, g->n[0], nullptr, F0, s));
  return EIFE_OK;
}

NormGeom make_norm_geom(const eife_grid_s* g, int pot = NORM_POT_DOUBLE_WELL) {
  NormGeom ng;
  ng.d = g->d;
  ng.cellvol = 1.0;
  ng.pot = pot;
  ng.th = g->c0;
  ng.thc = g->c1;
  for (int a = 0; a < 3; ++a) {
    ng.n[a] = g->n[a];
    ng.per[a] = g->per[a] ? 1 : 0;
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

// Block partial sums of the norm reduction into `partials` (at most
// kNormBlocksMax rows of kNormAcc doubles); returns the number of rows in *nb.
template <typename T>
int launch_norm_partials(eife_grid_s* g, const void* u, const void* uref, hipStream_t s, int pot, double* partials,
                         int* nb_out) {
  const NormGeom ng = make_norm_geom(g, pot);
  const int64_t total = int64_t(g->n[0]) * g->n[1] * g->n[2];
  const int64_t wpb = kNwThreads / 64;  // waves per block of the 3D reduction
  const int nxw = (g->n[0] + kNwOwn - 1) / kNwOwn;
  const int tiles_y = (g->n[1] + kNwRows - 1) / kNwRows;
  int nb;
  if (g->d == 3 && int64_t(nxw) * tiles_y <= wpb * kNormBlocksMax) {
    // 3D: waves of 62 x positions x 4 rows marching over z chunks (up to 16
    // chunks, as many as the partial rows allow; each also reads the plane
    // before it)
    const int nz = g->n[2];
    const int64_t fit = std::max<int64_t>(1, wpb * (kNormBlocksMax - 8) / (int64_t(nxw) * tiles_y));
    int nzc = int(std::max<int64_t>(1, std::min<int64_t>({int64_t(nz), 16, fit})));
    const int zc = (nz + nzc - 1) / nzc;
    nzc = (nz + zc - 1) / zc;
    const int64_t ntasks = int64_t(nxw) * tiles_y * nzc;
    nb = int(((ntasks + wpb - 1) / wpb + 7) / 8 * 8);
    if (nb > kNormBlocksMax) return fail(EIFE_EINVAL, "norm reduction needs %d partial rows (at most %d)", nb,
                                         kNormBlocksMax);
    const bool gen = ng.pot == NORM_POT_FH || ng.per[0] || ng.per[1] || ng.per[2];
    if (gen)
      hipLaunchKernelGGL((norm_waves<T, true>), dim3(nb), dim3(kNwThreads), 0, s, static_cast<const T*>(u),
                         static_cast<const T*>(uref), ng, zc, nxw, tiles_y, int(ntasks), partials);
    else
      hipLaunchKernelGGL((norm_waves<T, false>), dim3(nb), dim3(kNwThreads), 0, s, static_cast<const T*>(u),
                         static_cast<const T*>(uref), ng, zc, nxw, tiles_y, int(ntasks), partials);
  } else {
    nb = int(std::min<int64_t>(kNormBlocksMax, (total + kNormThreads - 1) / kNormThreads));
    nb = std::max(nb, 1);
    hipLaunchKernelGGL((norm_partial<T>), dim3(nb), dim3(kNormThreads), 0, s, static_cast<const T*>(u),
                       static_cast<const T*>(uref), ng, partials);
  }
  HIP_TRY(hipGetLastError());
  *nb_out = nb;
  return EIFE_OK;
}

template <typename T>
int run_norms(eife_grid_s* g, const void* u, const void* uref, hipStream_t s, int pot = NORM_POT_DOUBLE_WELL) {
  int nb = 0;
  RET_IF(launch_norm_partials<T>(g, u, uref, s, pot, g->partials, &nb));
  hipLaunchKernelGGL(norm_final, dim3(1), dim3(kNormFinalThreads), 0, s, g->partials, nb, g->out5);
  HIP_TRY(hipGetLastError());
  return EIFE_OK;
}

// Scratch of eife_norms_noalloc: the block partial rows of the reduction in a
// file-scope device array (320 KB on every GPU the library runs on, held until
// the process ends).  Host code never passes the array's name to a kernel: it
// uses the per-device address from hipGetSymbolAddress.  Calls that overlap on
// one GPU share the array and race.
static __device__ __align__(256) double scratch[kNormBlocksMax * kNormAcc];
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Address of the scratch array on `dev` (the current device), resolved once per device.
int scratch_on(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(EIFE_EUNSUPPORTED, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(EIFE_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<double*>(g_scratch_ptr[dev]);
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
  hipFree(g->X);
  for (int a = 0; a < 3; ++a) {
    hipFree(g->tw[a]);
    hipFree(g->tab[a]);
    hipFree(g->sinpi_ax[a]);
    hipFree(g->smat[a]);
  }
  for (auto& r : g->prof_pending) {
    g->ev_pool.push_back(r.a);
    g->ev_pool.push_back(r.b);
  }
  for (hipEvent_t e : g->ev_pool) hipEventDestroy(e);
  hipFree(g->partials);
  hipFree(g->out5);
  if (g->host5) hipHostFree(g->host5);
  hipFree(g->vtab);
  if (g->vhost) hipHostFree(g->vhost);
  for (int b = 0; b < 2; ++b)
    if (g->vev[b]) hipEventDestroy(g->vev[b]);
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
  if (bc != EIFE_BC_DIRICHLET && bc != EIFE_BC_PERIODIC) return fail(EIFE_EINVAL, "unknown boundary condition %d", bc);
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
    g->per[a] = bc == EIFE_BC_PERIODIC;
    g->n[a] = g->per[a] ? N[a] : N[a] - 1;
    g->h[a] = h[a];
  }
  for (int a = 0; a < 3; ++a) {
    // FFT length: the odd extension (2N) of a sine line, the line itself (N) when periodic
    if (!factor_plan(g->per[a] ? g->N[a] : 2 * g->N[a], &g->plan[a])) {
      const int bad = g->N[a];
      delete g;
      return fail(EIFE_EUNSUPPORTED, "N = %d: FFT length has more than three prime factors above 7", bad);
    }
  }
  g->pitch = ((g->n[0] + 31) / 32) * 32;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    delete g;
    return fail(EIFE_EHIP, "no HIP device");
  }
  g->device = dev;
  {
    double* sp = nullptr;  // the no-allocation reduction's scratch on this device, resolved at set-up
    if (scratch_on(dev, &sp) != EIFE_OK) {
      delete g;
      return EIFE_EHIP;
    }
  }
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
    if (hipMalloc(reinterpret_cast<void**>(&g->tab[a]), kTabArrays * size_t(g->tablen[a]) * sizeof(double)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&g->sinpi_ax[a]), size_t(g->n[a]) * sizeof(double)) != hipSuccess) {
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
  int rt = upload_tables(g);
  if (rt == EIFE_OK) rt = upload_sinpi(g);
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

int eife_set_nodes3(eife_grid g, double c2, double c3) {
  RET_IF(check_grid(g));
  if (!(c2 > 0.0 && c2 < c3 && c3 <= 1.0)) return fail(EIFE_EINVAL, "nodes must satisfy 0 < c2 < c3 <= 1");
  g->c2_3 = c2;
  g->c3_3 = c3;
  if (g->stages == 3) g->phi_ready = false;
  return EIFE_OK;
}

int eife_set_origin(eife_grid g, const double* a) {
  RET_IF(check_grid(g));
  if (!a) return fail(EIFE_EINVAL, "origin is null");
  for (int i = 0; i < g->d; ++i) {
    if (!std::isfinite(a[i])) return fail(EIFE_EINVAL, "origin must be finite");
    g->a[i] = a[i];
  }
  return upload_sinpi(g);
}

int eife_set_load(eife_grid g, int kind) {
  RET_IF(check_grid(g));
  if (kind != EIFE_LOAD_LUMPED && kind != EIFE_LOAD_NODAL) return fail(EIFE_EINVAL, "unknown load kind %d", kind);
  g->load = kind;
  return upload_tables(g);
}

int eife_set_transform(eife_grid g, int kind) {
  RET_IF(check_grid(g));
  if (kind != EIFE_TX_FFT && kind != EIFE_TX_FFT_GENERIC && kind != EIFE_TX_GEMM_SPLITBF16)
    return fail(EIFE_EINVAL, "unknown transform kind %d", kind);
  if (kind == EIFE_TX_GEMM_SPLITBF16) {
    if (g->dtype != EIFE_F32) return fail(EIFE_EUNSUPPORTED, "the split-BF16 transform takes FP32 grids only");
    if (g->per[0]) return fail(EIFE_EUNSUPPORTED, "the split-BF16 transform takes Dirichlet grids only");
    for (int a = 0; a < g->d; ++a)
      if (g->N[a] > 1024) return fail(EIFE_EUNSUPPORTED, "the split-BF16 transform takes N <= 1024 (N = %d)", g->N[a]);
    RET_IF(gemm_attrs_all());
    for (int a = 0; a < 3; ++a)
      if (!g->smat[a]) RET_IF(build_smat(g, a));
  }
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
  if (stages < 1 || stages > 3) return fail(EIFE_EINVAL, "stages must be 1, 2 or 3 (got %d)", stages);
  if (stages == 3 && !g->X) {
    const size_t bytes = size_t(g->pitch) * g->n[1] * g->n[2] * g->esz;
    if (hipMalloc(&g->X, bytes) != hipSuccess) {
      g->X = nullptr;
      return fail(EIFE_ENOMEM, "cannot allocate the three-stage state (%zu bytes)", bytes);
    }
    HIP_TRY(hipMemset(g->X, 0, bytes));
  }
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
  if (f_kind < EIFE_F_ZERO || f_kind > EIFE_F_TRAVELING_WAVE) return fail(EIFE_EINVAL, "unknown f_kind %d", f_kind);
  if (f_kind == EIFE_F_EX51 && g->d != 2) return fail(EIFE_EINVAL, "EIFE_F_EX51 is a 2D problem");
  if ((f_kind == EIFE_F_MMS_U2 || f_kind == EIFE_F_EX51 || f_kind == EIFE_F_TRAVELING_WAVE) && g->per[0])
    return fail(EIFE_EUNSUPPORTED, "f_kind %d is a Dirichlet problem", f_kind);
  if (f_kind == EIFE_F_TRAVELING_WAVE) {
    if (g->load != EIFE_LOAD_LUMPED)
      return fail(EIFE_EUNSUPPORTED, "boundary data enter the lumped load only (EIFE_LOAD_LUMPED)");
    if (!(g->c0 > 0.0)) return fail(EIFE_EINVAL, "EIFE_F_TRAVELING_WAVE needs eps = c0 > 0 (eife_set_forcing)");
  }
  if (!std::isfinite(t0)) return fail(EIFE_EINVAL, "t0 must be finite");
  if (!g->phi_ready) return fail(EIFE_ESTATE, "eife_set_phi must be called before eife_step");
  if (g->stages == 3 && g->transform == EIFE_TX_GEMM_SPLITBF16)
    return fail(EIFE_EUNSUPPORTED, "the three-stage scheme runs on the FFT transforms only");
  if (n_steps == 0) return EIFE_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (g->dtype == EIFE_F32)
    return run_steps<float>(g, static_cast<float*>(u), n_steps, f_kind, t0, s, nullptr, static_cast<float*>(u));
  return run_steps<double>(g, static_cast<double*>(u), n_steps, f_kind, t0, s, nullptr, static_cast<double*>(u));
}

int eife_step_out(eife_grid g, const void* u_in, void* u_out, int64_t n_steps, int f_kind, double t0,
                  void* stream) {
  if (!u_in || !u_out) return fail(EIFE_EINVAL, "u_in or u_out is null");
  if (n_steps < 0) return fail(EIFE_EINVAL, "n_steps must be >= 0");
  // the checks of eife_step (grid, f_kind, t0, state), without running anything
  RET_IF(eife_step(g, const_cast<void*>(u_in), 0, f_kind, t0, stream));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n_steps == 0) {
    const size_t bytes = size_t(g->n[0]) * g->n[1] * g->n[2] * g->esz;
    if (u_in != u_out) HIP_TRY(hipMemcpyAsync(u_out, u_in, bytes, hipMemcpyDeviceToDevice, s));
    return EIFE_OK;
  }
  if (g->dtype == EIFE_F32)
    return run_steps<float>(g, static_cast<const float*>(u_in), n_steps, f_kind, t0, s, nullptr,
                            static_cast<float*>(u_out));
  return run_steps<double>(g, static_cast<const double*>(u_in), n_steps, f_kind, t0, s, nullptr,
                           static_cast<double*>(u_out));
}

int eife_step_out_change(eife_grid g, const float* u_in, float* u_out, int64_t n_steps, int f_kind, double t0,
                         double* chg, int* done, void* stream) {
  if (!done) return fail(EIFE_EINVAL, "done is null");
  *done = 0;
  if (!u_in || !u_out || n_steps < 0) return fail(EIFE_EINVAL, "null u_in / u_out or negative n_steps");
  RET_IF(eife_step(g, const_cast<float*>(u_in), 0, f_kind, t0, stream));  // the checks of eife_step, nothing run
  if (n_steps < 1 || !chg || u_in == u_out || g->dtype != EIFE_F32 || !change_epilogue<float>(g))
    return eife_step_out(g, u_in, u_out, n_steps, f_kind, t0, stream);
  hipStream_t s = static_cast<hipStream_t>(stream);
  RET_IF(run_steps<float>(g, u_in, n_steps, f_kind, t0, s, nullptr, u_out, chg));
  *done = 1;
  return EIFE_OK;
}

int eife_step_variable(eife_grid g, void* u, const double* taus, int64_t n_steps, int f_kind, double t0,
                       void* stream) {
  RET_IF(check_grid(g));
  if (n_steps < 0) return fail(EIFE_EINVAL, "n_steps must be >= 0");
  if (n_steps > 0 && !taus) return fail(EIFE_EINVAL, "taus is null");
  for (int64_t i = 0; i < n_steps; ++i)
    if (!(taus[i] > 0.0) || !std::isfinite(taus[i]))
      return fail(EIFE_EINVAL, "taus[%lld] must be a positive finite number", static_cast<long long>(i));
  if (!g->phi_ready) return fail(EIFE_ESTATE, "eife_set_phi must be called before eife_step_variable");
  if (n_steps == 0) return eife_step(g, u, 0, f_kind, t0, stream);
  // the checks of eife_step on u, f_kind and t0, without running anything
  RET_IF(eife_step(g, u, 0, f_kind, t0, stream));
  RET_IF(ensure_step_tables(g));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (g->dtype == EIFE_F32)
    return run_steps<float>(g, static_cast<float*>(u), n_steps, f_kind, t0, s, taus, static_cast<float*>(u));
  return run_steps<double>(g, static_cast<double*>(u), n_steps, f_kind, t0, s, taus, static_cast<double*>(u));
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

int eife_norms_noalloc(eife_grid g, const void* u, const void* uref, double* out_dev, void* stream) {
  RET_IF(check_grid(g));
  if (!u || !out_dev) return fail(EIFE_EINVAL, "u and out_dev must not be null");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != g->device) return fail(EIFE_EINVAL, "the grid lives on device %d, the current device is %d", g->device, dev);
  double* part = nullptr;
  RET_IF(scratch_on(dev, &part));
  hipStream_t s = static_cast<hipStream_t>(stream);
  int nb = 0;
  RET_IF(g->dtype == EIFE_F32 ? launch_norm_partials<float>(g, u, uref, s, NORM_POT_DOUBLE_WELL, part, &nb)
                              : launch_norm_partials<double>(g, u, uref, s, NORM_POT_DOUBLE_WELL, part, &nb));
  double cellvol = 1.0;
  for (int a = 0; a < g->d; ++a) cellvol *= g->h[a];
  hipLaunchKernelGGL(norm_finish, dim3(1), dim3(kNormFinalThreads), 0, s, part, nb, g->D, cellvol, out_dev);
  HIP_TRY(hipGetLastError());
  return EIFE_OK;
}

int eife_energy(eife_grid g, const void* u, int f_kind, double* out, void* stream) {
  RET_IF(check_grid(g));
  if (!u || !out) return fail(EIFE_EINVAL, "u and out must not be null");
  int pot;
  if (f_kind == EIFE_F_ALLEN_CAHN)
    pot = NORM_POT_DOUBLE_WELL;
  else if (f_kind == EIFE_F_FLORY_HUGGINS)
    pot = NORM_POT_FH;
  else
    return fail(EIFE_EINVAL, "f_kind %d has no energy (Allen-Cahn or Flory-Huggins only)", f_kind);
  hipStream_t s = static_cast<hipStream_t>(stream);
  RET_IF(g->dtype == EIFE_F32 ? run_norms<float>(g, u, nullptr, s, pot) : run_norms<double>(g, u, nullptr, s, pot));
  HIP_TRY(hipMemcpyAsync(g->host5, g->out5, kNormAcc * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double cellvol = 1.0;
  for (int a = 0; a < g->d; ++a) cellvol *= g->h[a];
  out[0] = 0.5 * g->D * g->host5[3] + cellvol * g->host5[4];
  if (!std::isfinite(out[0])) return fail(EIFE_ENONFINITE, "energy is not finite");
  return EIFE_OK;
}

}  // extern "C"

// ===========================================================================
// Batches of independent 2D instances.
// ===========================================================================
struct eife_batch_s {
  int B = 0;
  int dtype = EIFE_F32;
  std::vector<eife_grid_s*> inst;
  std::vector<int64_t> uoff;  // B + 1 element offsets in the caller's array
  struct Class {
    std::vector<int> members;
    void* rinst = nullptr;    // RowInst<T>[members]
    void* cinst = nullptr;    // ColInst<T>[members], W -> H (stage passes)
    void* cinst_h = nullptr;  // ColInst<T>[members] acting on H only (prologue)
    int var_row = 0, var_col = 0;
    int prow = 0, pcol = 0;
  };
  std::vector<Class> classes;
  bool phi_ready = false;
  int stages = 0;
  // cached graph of the last captured step sequence
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  void* g_u = nullptr;
  int64_t g_steps = -1;
  int g_fkind = -1;
  double g_t0 = 0.0;
};

namespace {

template <typename T>
int build_batch_tables(eife_batch_s* b) {
  for (auto& c : b->classes) {
    const size_t n = c.members.size();
    std::vector<RowInst<T>> ri(n);
    std::vector<ColInst<T>> ci(n), ch(n);
    for (size_t k = 0; k < n; ++k) {
      eife_grid_s* g = b->inst[c.members[k]];
      ri[k].W = static_cast<T*>(g->W);
      ri[k].H = static_cast<T*>(g->H);
      ri[k].uoff = b->uoff[c.members[k]];
      ri[k].D = g->D;
      const Diag dg = make_diag(g);
      for (int a = 0; a < 3; ++a) ci[k].ax[a] = dg.ax[a];
      ci[k].W = static_cast<T*>(g->W);
      ci[k].H = static_cast<T*>(g->H);
      ci[k].D = g->D;
      ch[k] = ci[k];
      ch[k].W = static_cast<T*>(g->H);
    }
    if (hipMalloc(&c.rinst, n * sizeof(RowInst<T>)) != hipSuccess ||
        hipMalloc(&c.cinst, n * sizeof(ColInst<T>)) != hipSuccess ||
        hipMalloc(&c.cinst_h, n * sizeof(ColInst<T>)) != hipSuccess)
      return fail(EIFE_ENOMEM, "batch descriptor allocation failed");
    HIP_TRY(hipMemcpy(c.rinst, ri.data(), n * sizeof(RowInst<T>), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c.cinst, ci.data(), n * sizeof(ColInst<T>), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c.cinst_h, ch.data(), n * sizeof(ColInst<T>), hipMemcpyHostToDevice));
  }
  return EIFE_OK;
}

Batchlet class_batchlet(const eife_batch_s::Class& c, bool on_h) {
  Batchlet B;
  B.count = int(c.members.size());
  B.rinst = c.rinst;
  B.cinst = on_h ? c.cinst_h : c.cinst;
  B.var_row = c.var_row;
  B.var_col = c.var_col;
  B.prow = c.prow;
  B.pcol = c.pcol;
  return B;
}

// One EIFE step (both stages) of class c at time tn.
template <typename T>
int class_step(eife_batch_s* b, const eife_batch_s::Class& c, int f_kind, double tn, hipStream_t s,
               bool first_row_done = false) {
  eife_grid_s* g = b->inst[c.members[0]];
  const Batchlet B = class_batchlet(c, false);
  const Diag dg = make_diag(g);
  if (!first_row_done)
    RET_IF(launch_row<T>(g, ROW_PHYS, nullptr, g->pitch, nullptr, g->pitch, nullptr, make_forcing(g, f_kind, tn), s,
                         B));
  RET_IF(launch_col<T>(g, 1, g->stages == 1 ? COL_ETD1 : COL_STAGE_A, nullptr, nullptr, dg, s, B));
  if (g->stages == 2) {
    RET_IF(launch_row<T>(g, ROW_PHYS, nullptr, g->pitch, nullptr, g->pitch, nullptr,
                         make_forcing(g, f_kind, tn + g->c2 * g->tau), s, B));
    RET_IF(launch_col<T>(g, 1, COL_STAGE_B, nullptr, nullptr, dg, s, B));
  }
  return EIFE_OK;
}

template <typename T>
int batch_enqueue(eife_batch_s* b, T* u, int64_t n_steps, int f_kind, double t0, hipStream_t s) {
  for (auto& c : b->classes) {
    eife_grid_s* g = b->inst[c.members[0]];
    const Batchlet B = class_batchlet(c, false);
    const int mode = (n_steps > 0 && fused_first_row<T>(g, f_kind)) ? ROW_FWD_PHYS : ROW_FWD_USER;
    RET_IF(launch_row<T>(g, mode, u, g->n[0], nullptr, g->pitch, nullptr, make_forcing(g, f_kind, t0), s, B));
    RET_IF(launch_col<T>(g, 1, COL_PLAIN, nullptr, nullptr, make_diag(g), s, class_batchlet(c, true)));
  }
  for (int64_t st = 0; st < n_steps; ++st) {
    const double tn = t0 + double(st) * b->inst[0]->tau;
    for (auto& c : b->classes)
      RET_IF(class_step<T>(b, c, f_kind, tn, s, st == 0 && fused_first_row<T>(b->inst[c.members[0]], f_kind)));
  }
  for (auto& c : b->classes) {
    eife_grid_s* g = b->inst[c.members[0]];
    const Batchlet B = class_batchlet(c, false);
    RET_IF(launch_row<T>(g, ROW_INV_USER, nullptr, g->pitch, u, g->n[0], nullptr, make_forcing(g, f_kind, t0), s, B));
  }
  return EIFE_OK;
}

void drop_graph(eife_batch_s* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->g_steps = -1;
}

void free_batch(eife_batch_s* b) {
  if (!b) return;
  drop_graph(b);
  for (auto& c : b->classes) {
    (void)hipFree(c.rinst);
    (void)hipFree(c.cinst);
    (void)hipFree(c.cinst_h);
  }
  for (auto* g : b->inst) free_grid(g);
  delete b;
}

// --- autotuning -------------------------------------------------------------
std::string tune_key(const eife_batch_s* b, const eife_batch_s::Class& c) {
  const eife_grid_s* g = b->inst[c.members[0]];
  hipDeviceProp_t prop;
  char arch[64] = "gfx";
  if (hipGetDeviceProperties(&prop, g->device) == hipSuccess) snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
  for (char* p = arch; *p; ++p)
    if (*p == ':') *p = '_';
  char buf[256];
  snprintf(buf, sizeof(buf), "%s/%s/N%dx%d/n%zu", arch, b->dtype == EIFE_F32 ? "f32" : "f64", g->N[0], g->N[1],
           c.members.size());
  return buf;
}

// Cache file: a JSON object with one "key": [var_row, var_col, prow, pcol, us] entry per line.
bool tune_lookup(const char* path, const std::string& key, int v[4]) {
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    char k[256];
    int a, b2, c, d;
    double us;
    if (sscanf(line, " \"%255[^\"]\" : [ %d , %d , %d , %d , %lf ]", k, &a, &b2, &c, &d, &us) == 6 && key == k) {
      v[0] = a;
      v[1] = b2;
      v[2] = c;
      v[3] = d;
      found = true;
    }
  }
  fclose(f);
  return found;
}

void tune_store(const char* path, const std::string& key, const int v[4], double us) {
  if (!path) return;
  std::vector<std::string> entries;
  FILE* f = fopen(path, "r");
  if (f) {
    char line[512];
    while (fgets(line, sizeof(line), f)) {
      char k[256];
      if (sscanf(line, " \"%255[^\"]\"", k) == 1 && key != k) {
        std::string l(line);
        while (!l.empty() && (l.back() == '\n' || l.back() == ',' || l.back() == ' ')) l.pop_back();
        entries.push_back(l);
      }
    }
    fclose(f);
  }
  char buf[512];
  snprintf(buf, sizeof(buf), "  \"%s\": [%d, %d, %d, %d, %.3f]", key.c_str(), v[0], v[1], v[2], v[3], us);
  entries.push_back(buf);
  f = fopen(path, "w");
  if (!f) return;
  fprintf(f, "{\n");
  for (size_t i = 0; i < entries.size(); ++i) fprintf(f, "%s%s\n", entries[i].c_str(), i + 1 < entries.size() ? "," : "");
  fprintf(f, "}\n");
  fclose(f);
}

template <typename T>
int tune_class(eife_batch_s* b, eife_batch_s::Class& c, const char* path, hipStream_t s) {
  const std::string key = tune_key(b, c);
  eife_grid_s* g = b->inst[c.members[0]];
  const bool fast = g->transform == EIFE_TX_FFT && fast_len<T>(g->N[0]) && fast_len<T>(g->N[1]);
  const int ncol = sizeof(T) == 4 ? 4 : 2;  // FP32: also the pipelined stage pass
  // a launch shape this class can take: the specialised kernels' variants, or
  // line pairs per block whose LDS regions fit and whose tiles divide the pitch
  auto valid = [&](const std::array<int, 4>& cd) {
    if (fast) return cd[0] >= 0 && cd[0] < 2 && cd[1] >= 0 && cd[1] < ncol && cd[2] == 0 && cd[3] == 0;
    return cd[0] == 0 && cd[1] == 0 && cd[2] >= 1 && cd[3] >= 1 && cd[2] <= 64 && cd[3] <= 64 && pick_pairs(g, g->plan[0].L, cd[2]) == cd[2] &&
           pick_pairs(g, g->plan[1].L, cd[3]) == cd[3] && lds_bytes(g, cd[2], g->plan[0].L) <= 65536 &&
           lds_bytes(g, cd[3], g->plan[1].L) <= 65536 && g->pitch % (2 * cd[3]) == 0;
  };
  int v[4];
  if (tune_lookup(path, key, v) && valid({v[0], v[1], v[2], v[3]})) {
    c.var_row = v[0];
    c.var_col = v[1];
    c.prow = v[2];
    c.pcol = v[3];
    return EIFE_OK;
  }
  std::vector<std::array<int, 4>> cands;
  if (fast) {
    for (int r = 0; r < 2; ++r)
      for (int cc = 0; cc < ncol; ++cc) cands.push_back({r, cc, 0, 0});
  } else {
    for (int pr : {4, 8, 16})
      for (int pc : {4, 8, 16})
        if (valid({0, 0, pr, pc})) cands.push_back({0, 0, pr, pc});
  }
  if (cands.empty()) return EIFE_OK;  // no candidate fits: keep the defaults
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  double best = 1e30;
  std::array<int, 4> bestc = cands[0];
  for (const auto& cd : cands) {
    c.var_row = cd[0];
    c.var_col = cd[1];
    c.prow = cd[2];
    c.pcol = cd[3];
    RET_IF(class_step<T>(b, c, EIFE_F_ALLEN_CAHN, 0.0, s));  // warm
    HIP_TRY(hipEventRecord(e0, s));
    for (int r = 0; r < 3; ++r) RET_IF(class_step<T>(b, c, EIFE_F_ALLEN_CAHN, 0.0, s));
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) {
      best = ms;
      bestc = cd;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c.var_row = bestc[0];
  c.var_col = bestc[1];
  c.prow = bestc[2];
  c.pcol = bestc[3];
  const int vv[4] = {bestc[0], bestc[1], bestc[2], bestc[3]};
  tune_store(path, key, vv, best * 1e3 / 3.0);
  return EIFE_OK;
}

}  // namespace

extern "C" {

int eife_create_batch(int B, const int32_t* N, const double* h, const double* D, int dtype, eife_batch* out) {
  if (!out) return fail(EIFE_EINVAL, "out is null");
  *out = nullptr;
  if (B < 1 || !N || !h || !D) return fail(EIFE_EINVAL, "B must be >= 1 and N, h, D non-null");
  eife_batch_s* b = new eife_batch_s();
  b->B = B;
  b->dtype = dtype;
  b->uoff.assign(B + 1, 0);
  for (int i = 0; i < B; ++i) {
    eife_grid g = nullptr;
    const int r = eife_create_grid(2, N + 2 * i, h + 2 * i, D[i], EIFE_BC_DIRICHLET, dtype, &g);
    if (r != EIFE_OK) {
      const std::string msg = g_last_error;
      free_batch(b);
      return fail(r, "instance %d: %s", i, msg.c_str());
    }
    b->inst.push_back(g);
    b->uoff[i + 1] = b->uoff[i] + int64_t(g->n[0]) * g->n[1];
    // size class: equal N and h
    int found = -1;
    for (size_t k = 0; k < b->classes.size(); ++k) {
      const eife_grid_s* r0 = b->inst[b->classes[k].members[0]];
      if (r0->N[0] == g->N[0] && r0->N[1] == g->N[1] && r0->h[0] == g->h[0] && r0->h[1] == g->h[1]) found = int(k);
    }
    if (found < 0) {
      b->classes.emplace_back();
      found = int(b->classes.size()) - 1;
    }
    b->classes[found].members.push_back(i);
  }
  // default column variant before any tuning: FP32 classes of 512-interval
  // columns take the pipelined stage pass (measured faster)
  for (auto& c : b->classes) {
    const eife_grid_s* g0 = b->inst[c.members[0]];
    if (dtype == EIFE_F32 && g0->N[1] == 512 && g0->transform == EIFE_TX_FFT) c.var_col = 2;
  }
  const int r = dtype == EIFE_F32 ? build_batch_tables<float>(b) : build_batch_tables<double>(b);
  if (r != EIFE_OK) {
    free_batch(b);
    return r;
  }
  *out = b;
  return EIFE_OK;
}

int eife_destroy_batch(eife_batch b) {
  free_batch(b);
  return EIFE_OK;
}

int eife_batch_offsets(eife_batch b, int64_t* offsets) {
  if (!b || !offsets) return fail(EIFE_EINVAL, "null batch or offsets");
  for (int i = 0; i <= b->B; ++i) offsets[i] = b->uoff[i];
  return EIFE_OK;
}

int eife_batch_set_phi(eife_batch b, double tau, int stages) {
  if (!b) return fail(EIFE_EINVAL, "null batch");
  for (auto* g : b->inst) RET_IF(eife_set_phi(g, tau, stages));
  b->phi_ready = true;
  b->stages = stages;
  drop_graph(b);
  return EIFE_OK;
}

int eife_batch_step(eife_batch b, void* u, int64_t n_steps, int f_kind, double t0, void* stream) {
  if (!b) return fail(EIFE_EINVAL, "null batch");
  if (!u) return fail(EIFE_EINVAL, "u is null");
  if (n_steps < 0) return fail(EIFE_EINVAL, "n_steps must be >= 0");
  if (f_kind < EIFE_F_ZERO || f_kind > EIFE_F_AFFINE_T) return fail(EIFE_EINVAL, "unknown f_kind %d", f_kind);
  if (!std::isfinite(t0)) return fail(EIFE_EINVAL, "t0 must be finite");
  if (!b->phi_ready) return fail(EIFE_ESTATE, "eife_batch_set_phi must be called before eife_batch_step");
  if (n_steps == 0) return EIFE_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto enqueue = [&]() -> int {
    return b->dtype == EIFE_F32 ? batch_enqueue<float>(b, static_cast<float*>(u), n_steps, f_kind, t0, s)
                                : batch_enqueue<double>(b, static_cast<double*>(u), n_steps, f_kind, t0, s);
  };
  if (!s) return enqueue();  // the legacy default stream cannot be captured
  if (!(b->gexec && b->g_u == u && b->g_steps == n_steps && b->g_fkind == f_kind && b->g_t0 == t0)) {
    drop_graph(b);
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    const int r = enqueue();
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &graph);
    if (r != EIFE_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return r;
    }
    if (e != hipSuccess) return fail(EIFE_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    b->graph = graph;
    HIP_TRY(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
    b->g_u = u;
    b->g_steps = n_steps;
    b->g_fkind = f_kind;
    b->g_t0 = t0;
  }
  HIP_TRY(hipGraphLaunch(b->gexec, s));
  return EIFE_OK;
}

int eife_batch_autotune(eife_batch b, const char* cache_path, void* stream) {
  if (!b) return fail(EIFE_EINVAL, "null batch");
  if (!b->phi_ready) return fail(EIFE_ESTATE, "eife_batch_set_phi must be called before eife_batch_autotune");
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (auto& c : b->classes)
    RET_IF(b->dtype == EIFE_F32 ? tune_class<float>(b, c, cache_path, s) : tune_class<double>(b, c, cache_path, s));
  HIP_TRY(hipStreamSynchronize(s));
  drop_graph(b);
  return EIFE_OK;
}

int eife_batch_class_info(eife_batch b, int k, int32_t* out) {
  if (!b || !out) return fail(EIFE_EINVAL, "null batch or out");
  if (k < 0 || k >= int(b->classes.size())) return fail(EIFE_EINVAL, "class %d out of range", k);
  const auto& c = b->classes[k];
  const eife_grid_s* g = b->inst[c.members[0]];
  out[0] = g->N[0];
  out[1] = g->N[1];
  out[2] = int32_t(c.members.size());
  out[3] = c.prow > 0 ? c.prow : c.var_row;
  out[4] = c.pcol > 0 ? c.pcol : c.var_col;
  return EIFE_OK;
}

}  // extern "C"

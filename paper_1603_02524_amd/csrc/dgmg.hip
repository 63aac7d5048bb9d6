// C ABI of the gfx950 DG p-multigrid solver: handle, workspace, coarse solve,
// PCG vector kernels and the orchestration of Alg. 1 (V-cycle) and Alg. 2 (MGCG).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/dgmg.h"
#include "kernels.hpp"
#include "kernels_big.hpp"
#include "setup.hpp"

using namespace dgmg;

namespace dgmg {
extern template struct Kern<double, 3>;
extern template struct Kern<float, 3>;
extern template struct Kern<double, 2>;
extern template struct Kern<float, 2>;
}  // namespace dgmg

namespace {

thread_local std::string g_setup_error;

}  // namespace

// Message for dgmg_last_error(NULL) from the handle-free entry points of other
// translation units (the MLP kernels).
void dgmg_set_global_error(const std::string& msg) { g_setup_error = msg; }

namespace {

constexpr int RED_BLOCKS = 1024;  // fixed partial count of the vector reductions
constexpr int VEC_THREADS = 256;

// ---------------------------------------------------------------- vector kernels (FP64 PCG)
__global__ void __launch_bounds__(VEC_THREADS) k_dot(const double* __restrict__ a,
                                                     const double* __restrict__ b, int64_t n,
                                                     double* __restrict__ part, const int* act) {
  if (inactive(act)) return;
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += a[i] * b[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Sum of partials in a fixed order into out[0] (one block).
__global__ void __launch_bounds__(VEC_THREADS) k_finalize(const double* __restrict__ part, int np,
                                                          double* __restrict__ out, const int* act) {
  if (inactive(act)) return;
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = s;
}

// Phase-b scalars in one block: n = z.(r - r_old) and z.r from their partials
// (each in a fixed order), then beta = n / delta with the previous delta, and
// delta <- z.r; from now on r_old enters n with weight 1 (slot 6, 0 before the
// first direction update: r_old = 0 initially).  scal slots: 0 delta, 1 beta,
// 4 n, 5 z.r, 6 r_old weight.
__global__ void __launch_bounds__(VEC_THREADS) k_finalize_beta(const double* __restrict__ part1,
                                                               const double* __restrict__ part2, int np,
                                                               double* __restrict__ scal, const int* act) {
  if (inactive(act)) return;
  __shared__ double red[16];
  double s1 = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    s1 += part1[i];
    s2 += part2[i];
  }
  s1 = block_sum(s1, red);
  __syncthreads();
  s2 = block_sum(s2, red);
  if (threadIdx.x == 0) {
    scal[4] = s1;
    scal[5] = s2;
    scal[1] = s1 / scal[0];
    scal[0] = s2;
    scal[6] = 1.0;
  }
}

// sum a_i and sum |a_i| partials.
__global__ void __launch_bounds__(VEC_THREADS) k_sum_abs(const double* __restrict__ a, int64_t n,
                                                         double* __restrict__ part1,
                                                         double* __restrict__ part2, const int* act) {
  if (inactive(act)) return;
  __shared__ double red[16];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    s1 += a[i];
    s2 += fabs(a[i]);
  }
  s1 = block_sum(s1, red);
  __syncthreads();
  s2 = block_sum(s2, red);
  if (threadIdx.x == 0) {
    part1[blockIdx.x] = s1;
    part2[blockIdx.x] = s2;
  }
}

// z.(r - r_old) and z.r partials.  TZ = float: z is the FP32 V-cycle output,
// widened to FP64 as it is read (here and in k_update_p).
template <class TZ>
__global__ void __launch_bounds__(VEC_THREADS) k_dot_zr(const TZ* __restrict__ z,
                                                        const double* __restrict__ r,
                                                        const double* __restrict__ ro,
                                                        const double* __restrict__ ro_weight, int64_t n,
                                                        double* __restrict__ part1,
                                                        double* __restrict__ part2, const int* act) {
  if (inactive(act)) return;
  __shared__ double red[16];
  const double wo = ro_weight[0];  // 0 before the first direction update (r - 0 r_old = r exactly)
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double zi = (double)z[i], ri = r[i];
    s1 += zi * (ri - wo * ro[i]);
    s2 += zi * ri;
  }
  s1 = block_sum(s1, red);
  __syncthreads();
  s2 = block_sum(s2, red);
  if (threadIdx.x == 0) {
    part1[blockIdx.x] = s1;
    part2[blockIdx.x] = s2;
  }
}

// alpha = delta / (p.q); x += alpha p; r_old = r; r -= alpha q; partial r.r;
// rf (if not null) = r rounded to FP32, the input of the mixed-precision V-cycle
__global__ void __launch_bounds__(VEC_THREADS) k_update_xr(double* __restrict__ x, double* __restrict__ r,
                                                           double* __restrict__ ro,
                                                           const double* __restrict__ p,
                                                           const double* __restrict__ q,
                                                           const double* __restrict__ delta,
                                                           const double* __restrict__ pq, int64_t n,
                                                           double* __restrict__ part, float* __restrict__ rf,
                                                           const int* act) {
  if (inactive(act)) return;
  __shared__ double red[16];
  const double alpha = delta[0] / pq[0];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    const double r0 = r[i];
    ro[i] = r0;
    const double ri = r0 - alpha * q[i];
    r[i] = ri;
    if (rf) rf[i] = (float)ri;
    s += ri * ri;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// p = z + beta p (z FP64, or the FP32 V-cycle output widened)
template <class TZ>
__global__ void __launch_bounds__(VEC_THREADS) k_update_p(double* __restrict__ p, const TZ* __restrict__ z,
                                                          const double* __restrict__ beta_p,
                                                          int64_t n, const int* act) {
  if (inactive(act)) return;
  const double beta = beta_p[0];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    p[i] = (double)z[i] + beta * p[i];
  }
}

template <class A, class B>
__global__ void __launch_bounds__(VEC_THREADS) k_convert(const A* __restrict__ a, B* __restrict__ b, int64_t n, const int* act) {
  if (inactive(act)) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (B)a[i];
}

template <class T>
__global__ void __launch_bounds__(VEC_THREADS) k_fill(T* __restrict__ a, T v, int64_t n, const int* act) {
  if (inactive(act)) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// Deterministic pseudo-random values in [-1, 1) from the index (integer hash
// with the lowbias32 constants of C. Wellons), used as the probe right-hand side.
__global__ void __launch_bounds__(VEC_THREADS) k_fill_hash(double* __restrict__ a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t x = (uint32_t)i ^ (uint32_t)(i >> 32) ^ 0x9e3779b9u;
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    a[i] = (double)(x >> 8) * (1.0 / 8388608.0) - 1.0;
  }
}

__global__ void __launch_bounds__(VEC_THREADS) k_copy(const double* __restrict__ a, double* __restrict__ b, int64_t n, const int* act) {
  if (inactive(act)) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// a -= s[0] * scale
__global__ void __launch_bounds__(VEC_THREADS) k_sub_scalar(double* __restrict__ a, const double* __restrict__ s,
                                                            double scale, int64_t n, const int* act) {
  if (inactive(act)) return;
  const double v = s[0] * scale;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] -= v;
}

// g = M f with the tensor-product GLL mass (Sec. 2.4)
__global__ void __launch_bounds__(VEC_THREADS) k_mass(LevelDev<double> L, const double* __restrict__ f,
                                                      double* __restrict__ g) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.n_dof) return;
  const int NP = L.NP, dim = L.dim;
  const int NE = dim == 3 ? NP * NP * NP : NP * NP;
  const int e = (int)(q / NE), loc = (int)(q - (int64_t)e * NE);
  const int N1 = L.dir[0].N, N2 = L.dir[1].N;
  int m[3] = {e % N1, dim == 3 ? (e / N1) % N2 : e / N1, dim == 3 ? e / (N1 * N2) : 0};
  int ii[3] = {loc % NP, (loc / NP) % NP, dim == 3 ? loc / (NP * NP) : 0};
  double w = 1.0;
  for (int d = 0; d < dim; ++d) w *= L.dir[d].ecoef[m[d] * ECOEF_N + E_HALF_DX] * L.rho[ii[d]];
  g[q] = w * f[q];
}

// ---------------------------------------------------------------- coarse solve (global FDM, P = 1)
// One pass of the global fast-diagonalisation along direction d on the
// element-major P = 1 vector: out = (S_d^T or S_d) applied along d.
struct CoarseDev {
  int dim;
  int se;     // 1: continuous lattice vector (nl[d] nodes per direction)
  int nl[3];
  int N[3];
  const double* S[3];    // G_d x G_d row-major
  const double* lam[3];  // G_d
};

template <bool FWD, bool SCALE>
__global__ void __launch_bounds__(VEC_THREADS) k_coarse_pass(CoarseDev C, int d, const double* __restrict__ in,
                                                             double* __restrict__ out, int64_t n,
                                                             const int* act) {
  if (inactive(act)) return;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int dim = C.dim, NE = dim == 3 ? 8 : 4;
  const int e = (int)(q >> (dim == 3 ? 3 : 2)), loc = (int)(q & (NE - 1));
  const int N1 = C.N[0], N2 = C.N[1];
  int m[3] = {e % N1, dim == 3 ? (e / N1) % N2 : e / N1, dim == 3 ? e / (N1 * N2) : 0};
  int ii[3] = {loc & 1, (loc >> 1) & 1, (loc >> 2) & 1};
  const int G = 2 * C.N[d];
  const int I = 2 * m[d] + ii[d];
  const int64_t est = d == 0 ? NE : (d == 1 ? (int64_t)N1 * NE : (int64_t)N1 * N2 * NE);
  const int nst = 1 << d;
  const int64_t base = q - (int64_t)m[d] * est - ii[d] * nst;
  const double* S = C.S[d];
  double s = 0.0;
  // loads issued in groups of 8 ahead of the products (the sum keeps the order K = 0, 1, ...)
  int K = 0;
  for (; K + 8 <= G; K += 8) {
    double v[8], w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = K + u;
      v[u] = in[base + (int64_t)(k >> 1) * est + (k & 1) * nst];
      w[u] = FWD ? S[k * G + I] : S[I * G + k];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += w[u] * v[u];
  }
  for (; K < G; ++K) {
    const double v = in[base + (int64_t)(K >> 1) * est + (K & 1) * nst];
    s += (FWD ? S[K * G + I] : S[I * G + K]) * v;
  }
  if (SCALE) {
    double den = 0.0;
    for (int dd = 0; dd < dim; ++dd) den += C.lam[dd][2 * m[dd] + ii[dd]];
    s = den != 0.0 ? s / den : 0.0;
  }
  out[q] = s;
}

// The same pass on a continuous lattice vector (nl[d] nodes per direction,
// direction 1 fastest).
template <bool FWD, bool SCALE>
__global__ void __launch_bounds__(VEC_THREADS) k_coarse_pass_lat(CoarseDev C, int d, const double* __restrict__ in,
                                                                 double* __restrict__ out, int64_t n,
                                                                 const int* act) {
  if (inactive(act)) return;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int dim = C.dim;
  int s[3] = {0, 0, 0};
  int64_t rest = q;
  for (int e = 0; e < dim; ++e) {
    s[e] = (int)(rest % C.nl[e]);
    rest /= C.nl[e];
  }
  const int G = C.nl[d], I = s[d];
  const int64_t st = d == 0 ? 1 : (d == 1 ? (int64_t)C.nl[0] : (int64_t)C.nl[0] * C.nl[1]);
  const int64_t base = q - (int64_t)I * st;
  const double* S = C.S[d];
  double acc = 0.0;
  for (int K = 0; K < G; ++K) acc += (FWD ? S[(int64_t)K * G + I] : S[(int64_t)I * G + K]) * in[base + K * st];
  if (SCALE) {
    double den = 0.0;
    for (int dd = 0; dd < dim; ++dd) den += C.lam[dd][s[dd]];
    acc = den != 0.0 ? acc / den : 0.0;
  }
  out[q] = acc;
}

// g = M f on a continuous lattice (assembled GLL-lumped mass: per direction the
// sum over the elements sharing the node of (dx/2) rho_i).
__global__ void __launch_bounds__(VEC_THREADS) k_mass_se(LevelDev<double> L, const double* __restrict__ f,
                                                         double* __restrict__ g) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.n_dof) return;
  const int P = L.P;
  int64_t rest = q;
  double w = 1.0;
  for (int d = 0; d < L.dim; ++d) {
    const DirDev<double>& dd = L.dir[d];
    const int s = (int)(rest % dd.nl);
    rest /= dd.nl;
    const int gl = dd.periodic ? s : s + 1;
    const int m = gl / P, i = gl - m * P;
    double md;
    if (i != 0) md = dd.ecoef[m * ECOEF_N + E_HALF_DX] * L.rho[i];
    else {
      const int ml = m == 0 ? dd.N - 1 : m - 1;
      md = dd.ecoef[ml * ECOEF_N + E_HALF_DX] * L.rho[P] + dd.ecoef[m * ECOEF_N + E_HALF_DX] * L.rho[0];
    }
    w *= md;
  }
  g[q] = w * f[q];
}

inline unsigned vec_blocks(int64_t n) {
  int64_t b = (n + VEC_THREADS - 1) / VEC_THREADS;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

}  // namespace

// =================================================================== handle
constexpr int MAXL = 8;      // levels: P <= 32 gives at most 6
constexpr int NKIND = 4;     // sweep kinds: 0..2 face-centred normal d, 3 element-centred

struct dgmg_handle {
  SetupParams sp;
  dgmg_opts opts;
  std::vector<LevelHost> lv;
  hipStream_t stream = nullptr;
  std::string err;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0, ws_need = 0;
  bool bound = false;
  std::vector<LevelDev<double>> Ld;
  std::vector<LevelDev<float>> Lf;
  struct Bufs {
    void* u = nullptr;
    void* f = nullptr;
    void* r = nullptr;
  };
  std::vector<Bufs> buf;  // per level, multigrid precision (r sized for doubles)
  void* patch = nullptr;  // patch buffer (sized for doubles)
  size_t patch_elems = 0;
  double *c_a = nullptr, *c_b = nullptr, *c_f = nullptr;  // coarse FDM scratch
  CoarseDev cdev{};
  // PCG (top level, FP64)
  double *pr = nullptr, *pro = nullptr, *pp = nullptr, *pq = nullptr, *pz = nullptr;
  double *part = nullptr, *part2 = nullptr;  // reduction partials
  double* scal = nullptr;                    // slots: 0 delta, 1 beta, 2 p.q, 3 r.r, 4 z.(r-r_old), 5 z.r, 6 r_old weight
  double* host_scal = nullptr;               // pinned
  // batched use: device flag (kernels return when 0) and the slot receiving r.r
  const int* active = nullptr;
  double* rr_out = nullptr;
  // hipGraph replay of the PCG phases
  bool use_graphs = false;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  const double* graph_x = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream used only while capturing
  // per-face (theta, omega) of the face-centred normal weights; empty = the fixed weights
  std::vector<double> face_theta, face_omega;
  // multiplicative smoothers: per level and sweep kind the patch launches of
  // one forward sweep, in order (colour classes, or single patches in
  // lexicographic order)
  struct MultClass {
    PatchLat lat;
    int n[3] = {1, 1, 1};
  };
  std::vector<MultClass> mcls[MAXL][NKIND];
  // autotuned patch-solve block shapes (waves per block), 0 = default
  int waves[MAXL][NKIND] = {};
  float tune_ms[MAXL][NKIND] = {};
  // timing of the top-level patch solves: every timing_stride-th launch
  // (counted in timing_count) carries an event pair
  bool timing = false;
  int timing_stride = 1;
  int64_t timing_count = 0;
  // V-cycle residual + restriction in one launch where built; the environment
  // variable DGMG_NO_FUSED_RESTRICTION at setup selects the two-step path
  // (same values; kept for comparison)
  bool fuse_restrict = true;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;  // recorded, not yet read
  std::vector<hipEvent_t> ev_pool;                       // created once, reused
  std::vector<double> ev_flops, ev_bytes;
  double t_ms = 0, t_flops = 0, t_bytes = 0;
  int64_t t_launch = 0;
};

struct dgmg_batch {
  std::vector<dgmg_handle*> h;
  std::vector<size_t> sub_off;
  std::vector<int64_t> dof_off;
  size_t ws_need = 0;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int* flags_dev = nullptr;
  double* rr_dev = nullptr;
  int* flags_host = nullptr;
  double* rr_host = nullptr;
  bool bound = false;
  // graph replay of the phases (off by default: an eager planned phase can
  // leave out the per-grid operations of converged grids, a recorded one
  // cannot, and measured faster on the 64-grid workload)
  bool use_graphs = false;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  const double* graph_x = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream used only while capturing
  std::string err;
  // batched execution plan (see batch_plan): per MGCG phase the launches over
  // work lists of all grids; descriptors in the workspace at plan_off
  struct Launch {
    int kind = 0, dim = 3, f32 = 0, t[4] = {0, 0, 0, 0};
    int ng = 0, ntot = 0;
    size_t desc_off = 0, starts_off = 0;
    std::vector<std::function<int()>> fns;
    std::vector<int> fn_grid;  // the grid of each of fns
    std::vector<int> key;      // plan position (launches of one position touch disjoint grids)
  };
  bool planned = false;
  std::vector<Launch> plan[2];
  // the per-grid steps of one plan position run on NSIDE side streams at once
  // (forked from and joined back into the phase's stream with events)
  // Used when the batch holds a grid whose top level fills the GPU alone
  // (measured: the 64-grid workload 376 -> 364 ms; a batch of small grids only
  // slowed down, 38.0 -> 41.4 ms, its steps too short for the fork and join).
  static constexpr int NSIDE = 3;
  hipStream_t side[NSIDE] = {};
  hipEvent_t ev_fork = nullptr, ev_join[NSIDE] = {};
  int nside = 0;
  bool concurrent = false;
  size_t plan_off = 0, plan_bytes = 0;
  double* x_cur = nullptr;  // the solve's x while a phase is recorded or run
};

namespace {

int fail(dgmg_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  else g_setup_error = msg;
  return code;
}

int check_hip(dgmg_handle* h, const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(h, DGMG_EHIP, std::string(where) + ": " + hipGetErrorString(e));
  return DGMG_OK;
}

bool mixed(const dgmg_handle* h) { return h->opts.precision == DGMG_PREC_MIXED; }
bool ec_smoother(const dgmg_handle* h) {
  return h->opts.smoother == DGMG_SMOOTHER_EA || h->opts.smoother == DGMG_SMOOTHER_EM;
}
bool multiplicative(const dgmg_handle* h) {
  return h->opts.smoother == DGMG_SMOOTHER_EM || h->opts.smoother == DGMG_SMOOTHER_FM;
}

// Patch launches of one forward multiplicative sweep (Sec. 3.1) on a level,
// normal nd (-1: element-centred).  Per direction the patch indices are split
// into groups: ORDER_LEX one group per patch (the lexicographic order,
// direction 0 fastest); ORDER_COLOUR the residues mod k (k = 2 along the
// face-centred normal and without overlap, 3 with overlap: patches k apart
// share no node and no matrix entry) followed, on a periodic direction whose
// count is not a multiple of k, by the last count mod k patches one by one.
// A launch is one group per direction; launches run with direction 0's group
// fastest.
std::vector<dgmg_handle::MultClass> mult_classes(const LevelHost& lv, int nd, int order) {
  struct Grp {
    int start, stride, count;
  };
  std::vector<Grp> grp[3];
  for (int d = 0; d < 3; ++d) {
    if (d >= lv.dim) {
      grp[d].push_back({0, 1, 1});
      continue;
    }
    const Dir1D& s = lv.dir[d];
    const int cnt = d == nd ? s.nf : s.N;
    if (order == DGMG_ORDER_LEX) {
      for (int c = 0; c < cnt; ++c) grp[d].push_back({c, 1, 1});
      continue;
    }
    const int k = (d == nd || lv.NO == 0) ? 2 : 3;
    const int rem = s.periodic ? cnt % k : 0;
    for (int j = 0; j < k; ++j) {
      const int m = (cnt - rem - j + k - 1) / k;
      if (m > 0) grp[d].push_back({j, k, m});
    }
    for (int i = 0; i < rem; ++i) grp[d].push_back({cnt - rem + i, 1, 1});
  }
  std::vector<dgmg_handle::MultClass> out;
  for (const Grp& g2 : grp[2])
    for (const Grp& g1 : grp[1])
      for (const Grp& g0 : grp[0]) {
        dgmg_handle::MultClass c;
        const Grp* g[3] = {&g0, &g1, &g2};
        for (int d = 0; d < 3; ++d) {
          c.lat.start[d] = g[d]->start;
          c.lat.stride[d] = g[d]->stride;
          c.n[d] = g[d]->count;
        }
        out.push_back(c);
      }
  return out;
}
size_t mg_size(const dgmg_handle* h) { return mixed(h) ? sizeof(float) : sizeof(double); }

// Workspace carving: a dry run (base == nullptr) computes the size.
struct Carver {
  char* base;
  size_t off = 0;
  void* take(size_t bytes) {
    off = (off + 255) & ~size_t(255);
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

using Upload = std::vector<std::pair<void*, std::vector<char>>>;

template <class T>
void carve_level(Carver& cv, const LevelHost& h, LevelDev<T>& d, Upload* up) {
  auto put = [&](const std::vector<double>& v) -> const T* {
    void* p = cv.take(v.size() * sizeof(T));
    if (up && p) {
      std::vector<char> bytes(v.size() * sizeof(T));
      T* t = reinterpret_cast<T*>(bytes.data());
      for (size_t i = 0; i < v.size(); ++i) t[i] = (T)v[i];
      up->emplace_back(p, std::move(bytes));
    }
    return (const T*)p;
  };
  auto put_int = [&](const std::vector<int>& v) -> const int* {
    void* p = cv.take(v.size() * sizeof(int));
    if (up && p) {
      std::vector<char> bytes(v.size() * sizeof(int));
      std::memcpy(bytes.data(), v.data(), bytes.size());
      up->emplace_back(p, std::move(bytes));
    }
    return (const int*)p;
  };
  auto transp = [](const std::vector<double>& S, int n) {
    std::vector<double> t(S.size());
    const size_t nb = S.size() / ((size_t)n * n);
    for (size_t b = 0; b < nb; ++b)
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) t[b * n * n + (size_t)j * n + i] = S[b * n * n + (size_t)i * n + j];
    return t;
  };
  // gather offsets of every patch position into the level vector (element-major)
  auto offsets = [&](int dir, int npatch, int len, bool fc) {
    const Dir1D& s = h.dir[dir];
    const int NP = h.NP, G = s.N * NP;
    int64_t NE = 1;
    for (int e = 0; e < h.dim; ++e) NE *= NP;
    int64_t est = NE;
    for (int e = 0; e < dir; ++e) est *= h.dir[e].N;
    int64_t nst = 1;
    for (int e = 0; e < dir; ++e) nst *= NP;
    std::vector<int> t((size_t)npatch * len);
    if (h.se) {  // lattice vectors: patch q's tile starts at lattice position q P - N_O
      int64_t lst = 1;
      for (int e = 0; e < dir; ++e) lst *= h.dir[e].nl;
      const int NT = s.N * h.P;
      for (int q = 0; q < npatch; ++q)
        for (int o = 0; o < len; ++o) {
          const int g = q * h.P - h.NO + o;
          int st = -1;
          if (s.periodic) st = ((g % NT) + NT) % NT;
          else if (g >= 1 && g <= NT - 1) st = g - 1;
          t[(size_t)q * len + o] = st < 0 ? -1 : (int)(st * lst);
        }
      return t;
    }
    for (int q = 0; q < npatch; ++q)
      for (int o = 0; o < len; ++o) {
        int g = (fc ? (q - 1) * NP + 1 : q * NP - h.NO) + o;
        if (s.periodic) g = ((g % G) + G) % G;
        int off = -1;
        if (g >= 0 && g < G) off = (int)((g / NP) * est + (g % NP) * nst);
        t[(size_t)q * len + o] = off;
      }
    return t;
  };
  d.dim = h.dim;
  d.se = h.se ? 1 : 0;
  d.P = h.P;
  d.NP = h.NP;
  d.NO = h.NO;
  d.NPc = h.NPc;
  d.n_elem = (int)h.n_elem;
  d.n_dof = h.n_dof;
  d.Ls = put(h.Ls);
  d.D = put(h.D);
  d.rho = put(h.rho);
  d.J = h.J.empty() ? nullptr : put(h.J);
  for (int k = 0; k < 3; ++k) {
    DirDev<T>& dd = d.dir[k];
    dd = DirDev<T>();
    if (k >= h.dim) continue;
    const Dir1D& s = h.dir[k];
    dd.N = s.N;
    dd.periodic = s.periodic;
    dd.nl = s.nl;
    dd.n_ec = s.n_ec;
    dd.n_fc = s.n_fc;
    dd.nf = s.nf;
    dd.ecoef = put(s.ecoef);
    dd.nbr = put_int(s.nbr);
    if (!s.S_ec.empty()) {
      dd.S_ec = put(s.S_ec);
      dd.ST_ec = put(transp(s.S_ec, s.n_ec));
      dd.lam_ec = put(s.lam_ec);
      dd.w_ec = put(s.w_ec);
      if (!h.se) {  // continuous levels have element-centred subdomains only
        dd.S_fc = put(s.S_fc);
        dd.ST_fc = put(transp(s.S_fc, s.n_fc));
        dd.lam_fc = put(s.lam_fc);
        dd.w_fc = put(s.w_fc);
      }
      dd.goff_ec = put_int(offsets(k, s.N, s.n_ec, false));
      if (!h.se) dd.goff_fc = put_int(offsets(k, s.nf, s.n_fc, true));
    }
  }
}

// Patch-buffer elements needed by one sweep with normal direction nd on a level.
size_t sweep_patch_elems(const LevelHost& lv, int nd) {
  size_t np = 1, ts = 1;
  for (int d = 0; d < lv.dim; ++d) {
    const Dir1D& s = lv.dir[d];
    const bool fc = d == nd;
    np *= fc ? s.nf : s.N;
    ts *= fc ? s.n_fc : s.n_ec;
  }
  return np * ts;
}

void layout(dgmg_handle* h, char* base, Upload* up) {
  Carver cv{base};
  const int nl = (int)h->lv.size();
  h->Ld.assign(nl, LevelDev<double>());
  h->Lf.assign(nl, LevelDev<float>());
  for (int l = 0; l < nl; ++l) {
    carve_level<double>(cv, h->lv[l], h->Ld[l], up);
    carve_level<float>(cv, h->lv[l], h->Lf[l], up);
  }
  const LevelHost& l0 = h->lv[0];
  h->cdev.dim = l0.dim;
  h->cdev.se = l0.se ? 1 : 0;
  for (int d = 0; d < 3; ++d) {
    h->cdev.N[d] = d < l0.dim ? l0.dir[d].N : 1;
    h->cdev.nl[d] = d < l0.dim ? l0.dir[d].nl : 1;
    if (d >= l0.dim) continue;
    const Dir1D& s = l0.dir[d];
    void* pS = cv.take(s.S_glob.size() * sizeof(double));
    void* pl = cv.take(s.lam_glob.size() * sizeof(double));
    if (up && pS) {
      std::vector<char> b1(s.S_glob.size() * 8), b2(s.lam_glob.size() * 8);
      std::memcpy(b1.data(), s.S_glob.data(), b1.size());
      std::memcpy(b2.data(), s.lam_glob.data(), b2.size());
      up->emplace_back(pS, std::move(b1));
      up->emplace_back(pl, std::move(b2));
    }
    h->cdev.S[d] = (const double*)pS;
    h->cdev.lam[d] = (const double*)pl;
  }
  const size_t es = mg_size(h);
  h->buf.assign(nl, dgmg_handle::Bufs());
  size_t pmax = 0;
  for (int l = 0; l < nl; ++l) {
    const size_t n = h->lv[l].n_dof;
    h->buf[l].u = cv.take(n * es);
    h->buf[l].f = cv.take(n * es);
    h->buf[l].r = cv.take(n * std::max<size_t>(es, sizeof(double)));
    if (l > 0) {
      pmax = std::max(pmax, sweep_patch_elems(h->lv[l], -1));
      for (int d = 0; d < h->lv[l].dim; ++d) pmax = std::max(pmax, sweep_patch_elems(h->lv[l], d));
    }
  }
  pmax = std::max(pmax, (size_t)l0.n_dof);
  for (int l = 0; l < nl; ++l)  // continuous levels: element-major copies of the apply and restriction
    if (h->lv[l].se) {
      size_t ne = (size_t)h->lv[l].n_elem;
      for (int d = 0; d < h->lv[l].dim; ++d) ne *= h->lv[l].NP;
      pmax = std::max(pmax, ne);
    }
  for (int l = 1; l < nl; ++l)  // scratch of the transfers and the apply of large 3D elements
    if (h->lv[l].dim == 3 && h->lv[l].NP == BIG_NP) {
      pmax = std::max(pmax, (size_t)transfer_big_scratch((int)h->lv[l].n_elem, h->lv[l].NP, h->lv[l].NPc));
      pmax = std::max(pmax, (size_t)apply_big_scratch((int)h->lv[l].n_elem, h->lv[l].NP));
    }
  h->patch_elems = pmax;
  h->patch = cv.take(pmax * sizeof(double));
  const size_t n0 = l0.n_dof;
  h->c_a = (double*)cv.take(n0 * 8);
  h->c_b = (double*)cv.take(n0 * 8);
  h->c_f = (double*)cv.take(n0 * 8);
  const size_t nt = h->lv.back().n_dof;
  h->pr = (double*)cv.take(nt * 8);
  h->pro = (double*)cv.take(nt * 8);
  h->pp = (double*)cv.take(nt * 8);
  h->pq = (double*)cv.take(nt * 8);
  h->pz = (double*)cv.take(nt * 8);
  // partial sums of the MODE-2 apply: one per block (several per element on large 3D elements)
  const LevelHost& top = h->lv.back();
  const size_t per_elem =
      (top.dim == 3 && top.NP == BIG_NP) ? (size_t)apply_big_blocks_per_elem<double, BIG_NP>() : 1;  // FP64: most blocks
  const size_t np1 = std::max<size_t>(RED_BLOCKS, top.n_elem * per_elem + 8);
  h->part = (double*)cv.take(np1 * 8);
  h->part2 = (double*)cv.take(RED_BLOCKS * 8);
  h->scal = (double*)cv.take(64 * 8);
  h->ws_need = cv.off + 256;
  for (int l = 0; l < nl; ++l) {
    h->Ld[l].active = h->active;
    h->Lf[l].active = h->active;
  }
}

// ---------------------------------------------------------------- typed level operations
template <class T>
const LevelDev<T>& LD(dgmg_handle* h, int l);
template <>
const LevelDev<double>& LD<double>(dgmg_handle* h, int l) { return h->Ld[l]; }
template <>
const LevelDev<float>& LD<float>(dgmg_handle* h, int l) { return h->Lf[l]; }

template <class T>
int k_apply(dgmg_handle* h, int l, int mode, const T* x, const T* f, T* y, double* part, int* nb) {
  const LevelDev<T>& L = LD<T>(h, l);
  T* scratch = (T*)h->patch;  // idle outside the patch solves of a sweep
  if (L.se) {  // element copies into the patch buffer, then the node sums
    const int m = mode == 2 ? 0 : mode;
    int rc = L.dim == 3 ? Kern<T, 3>::se_apply(L, m, x, f, y, scratch, h->stream)
                        : Kern<T, 2>::se_apply(L, m, x, f, y, scratch, h->stream);
    if (rc) return fail(h, DGMG_EUNSUPPORTED, "no continuous operator kernel for this order");
    if (mode == 2) {  // partial sums of x.y for the PCG
      if constexpr (std::is_same<T, double>::value) {
        hipLaunchKernelGGL(k_dot, dim3(RED_BLOCKS), dim3(VEC_THREADS), 0, h->stream, x, y, L.n_dof, part, h->active);
        *nb = RED_BLOCKS;
      } else {
        return fail(h, DGMG_EINVAL, "mode 2 is FP64 only");
      }
    }
    return check_hip(h, "apply");
  }
  const bool comp = L.dim == 3 ? Kern<T, 3>::order_compiled(L.NP) : Kern<T, 2>::order_compiled(L.NP);
  if (!comp && mode == 2) {  // run-time orders: the operator, then the partial sums of x.y
    int rc = L.dim == 3 ? Kern<T, 3>::apply(L, 0, x, f, y, scratch, part, nb, h->stream)
                        : Kern<T, 2>::apply(L, 0, x, f, y, scratch, part, nb, h->stream);
    if (rc) return fail(h, DGMG_EUNSUPPORTED, "no operator kernel for this order");
    if constexpr (std::is_same<T, double>::value) {
      hipLaunchKernelGGL(k_dot, dim3(RED_BLOCKS), dim3(VEC_THREADS), 0, h->stream, x, y, L.n_dof, part, h->active);
      *nb = RED_BLOCKS;
      return check_hip(h, "apply");
    } else {
      return fail(h, DGMG_EINVAL, "mode 2 is FP64 only");
    }
  }
  int rc = L.dim == 3 ? Kern<T, 3>::apply(L, mode, x, f, y, scratch, part, nb, h->stream)
                      : Kern<T, 2>::apply(L, mode, x, f, y, scratch, part, nb, h->stream);
  if (rc) return fail(h, DGMG_EUNSUPPORTED, "no operator kernel for this order");
  return check_hip(h, "apply");
}

void sweep_shape(const LevelHost& lv, int nd, int np[3], int& NA, int& NL) {
  np[0] = np[1] = np[2] = 1;
  for (int d = 0; d < lv.dim; ++d) np[d] = (d == nd) ? lv.dir[d].nf : lv.dir[d].N;
  NL = lv.NP + 2 * lv.NO;
  NA = nd < 0 ? NL : 2 * lv.P;
}

template <class T>
int k_fdm(dgmg_handle* h, int l, int nd, const T* r, int waves) {
  const LevelDev<T>& L = LD<T>(h, l);
  int np[3], NA, NL;
  sweep_shape(h->lv[l], nd, np, NA, NL);
  T* pb = (T*)h->patch;
  const PatchLat all;
  int rc = L.dim == 3 ? Kern<T, 3>::fdm(L, nd, NA, NL, r, pb, np[0], np[1], np[2], waves, all, h->stream)
                      : Kern<T, 2>::fdm(L, nd, NA, NL, r, pb, np[0], np[1], np[2], waves, all, h->stream);
  if (rc) return fail(h, DGMG_EUNSUPPORTED, "no patch-solve kernel for this tile");
  return DGMG_OK;
}

// One additive sweep.  u_zero: the caller guarantees u == 0, so the residual
// f - A u is f itself and the patch solves read f directly.
// Timing events: taken from a pool created when timing is enabled (no event
// creation inside a timed region), returned to it once read.
hipEvent_t take_event(dgmg_handle* h) {
  if (h->ev_pool.empty()) {
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  hipEvent_t e = h->ev_pool.back();
  h->ev_pool.pop_back();
  return e;
}

template <class T>
int k_sweep(dgmg_handle* h, int l, int nd, T* u, const T* f, T* r, bool u_zero = false) {
  const LevelDev<T>& L = LD<T>(h, l);
  const LevelHost& lv = h->lv[l];
  int rc = u_zero ? DGMG_OK : k_apply<T>(h, l, 1, u, f, r, nullptr, nullptr);
  if (rc) return rc;
  const T* res = u_zero ? f : r;
  int np[3], NA, NL;
  sweep_shape(lv, nd, np, NA, NL);
  const int kind = nd < 0 ? 3 : nd;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  // top-level launches only, every timing_stride-th of them
  const bool timed = h->timing && l == (int)h->lv.size() - 1 && (h->timing_count++ % h->timing_stride) == 0;
  if (timed) {
    e0 = take_event(h);
    e1 = take_event(h);
    (void)hipEventRecord(e0, h->stream);
  }
  rc = k_fdm<T>(h, l, nd, res, h->waves[l][kind]);
  if (rc) return rc;
  if (timed) {
    (void)hipEventRecord(e1, h->stream);
    h->ev.emplace_back(e0, e1);
    // algorithmic cost of one launch: 2 flops per multiply-add of the forward
    // and backward 1D contractions plus the scale and the weight; bytes: the
    // residual tile read and the weighted correction written, per patch
    const double npatch = (double)np[0] * np[1] * np[2];
    double ts = NA;
    for (int d = 1; d < lv.dim; ++d) ts *= NL;
    const double fl = 2.0 * 2.0 * ts * (NA + (lv.dim - 1) * NL) + 2.0 * ts;
    h->ev_flops.push_back(npatch * fl);
    h->ev_bytes.push_back(npatch * ts * 2.0 * sizeof(T));
  }
  rc = check_hip(h, "patch solve");
  if (rc) return rc;
  T* pb = (T*)h->patch;
  // u == 0 on entry: the overlap sum is assigned (no fill of u beforehand, no read of it)
  if (L.se)
    rc = L.dim == 3 ? Kern<T, 3>::se_combine(L, NA, pb, u, u_zero, h->stream)
                    : Kern<T, 2>::se_combine(L, NA, pb, u, u_zero, h->stream);
  else
    rc = L.dim == 3 ? Kern<T, 3>::combine(L, nd, NA, NL, pb, u, np[0], np[1], np[2], u_zero, h->stream)
                    : Kern<T, 2>::combine(L, nd, NA, NL, pb, u, np[0], np[1], np[2], u_zero, h->stream);
  if (rc) return fail(h, DGMG_EUNSUPPORTED, "no combine kernel for this order");
  return check_hip(h, "combine");
}

template <class T>
void k_fill_v(dgmg_handle* h, T* a, int64_t n, T v = T(0)) {
  hipLaunchKernelGGL(k_fill<T>, dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, a, v, n, h->active);
}

// One multiplicative sweep (Sec. 3.1): the patch launches of the level's
// order (reversed when `reverse`), each on the residual left by the previous
// ones: r = f - A u, the launch's patch solves, u += their corrections
// (unweighted; the weight tables of a multiplicative handle are 1).
// u_zero: u is taken as 0 on entry (it is cleared; the first launch reads f).
template <class T>
int k_msweep(dgmg_handle* h, int l, int nd, T* u, const T* f, T* r, bool reverse, bool u_zero) {
  const LevelDev<T>& L = LD<T>(h, l);
  const LevelHost& lv = h->lv[l];
  int np[3], NA, NL;
  sweep_shape(lv, nd, np, NA, NL);
  const int kind = nd < 0 ? 3 : nd;
  const auto& cls = h->mcls[l][kind];
  if (u_zero) k_fill_v<T>(h, u, lv.n_dof);
  T* pb = (T*)h->patch;
  const int nc = (int)cls.size();
  for (int i = 0; i < nc; ++i) {
    const dgmg_handle::MultClass& c = cls[reverse ? nc - 1 - i : i];
    const bool first = u_zero && i == 0;
    int rc = first ? DGMG_OK : k_apply<T>(h, l, 1, u, f, r, nullptr, nullptr);
    if (rc) return rc;
    const T* res = first ? f : r;
    rc = L.dim == 3
             ? Kern<T, 3>::fdm(L, nd, NA, NL, res, pb, c.n[0], c.n[1], c.n[2], h->waves[l][kind], c.lat, h->stream)
             : Kern<T, 2>::fdm(L, nd, NA, NL, res, pb, c.n[0], c.n[1], c.n[2], h->waves[l][kind], c.lat, h->stream);
    if (rc) return fail(h, DGMG_EUNSUPPORTED, "no patch-solve kernel for this multiplicative sweep");
    rc = L.dim == 3 ? Kern<T, 3>::mult_update(L, nd, NA, NL, c.lat, c.n[0], c.n[1], c.n[2], pb, u, h->stream)
                    : Kern<T, 2>::mult_update(L, nd, NA, NL, c.lat, c.n[0], c.n[1], c.n[2], pb, u, h->stream);
    if (rc) return fail(h, DGMG_EUNSUPPORTED, "multiplicative update");
  }
  return check_hip(h, "multiplicative sweep");
}

// `steps` smoothing steps (EA: one sweep; FA: one sweep per direction).
// Multiplicative (EM, FM): within the call every second step runs backwards
// (reversed patch order and, FM, reversed sweep directions), so that an even
// number of steps is symmetric (Sec. 3.1).
// u_zero: u is taken as 0 on entry, whatever it holds (the first sweep skips
// its residual apply and assigns u); needs steps >= 1.
template <class T>
int k_smooth(dgmg_handle* h, int l, T* u, const T* f, int steps, T* r, bool u_zero = false) {
  if (multiplicative(h)) {
    const int dim = h->lv[l].dim;
    for (int s = 0; s < steps; ++s) {
      const bool rev = s % 2 == 1;
      if (ec_smoother(h)) {
        int rc = k_msweep<T>(h, l, -1, u, f, r, rev, u_zero && s == 0);
        if (rc) return rc;
        continue;
      }
      for (int i = 0; i < dim; ++i) {
        int rc = k_msweep<T>(h, l, rev ? dim - 1 - i : i, u, f, r, rev, u_zero && s == 0 && i == 0);
        if (rc) return rc;
      }
    }
    return DGMG_OK;
  }
  for (int s = 0; s < steps; ++s) {
    if (h->opts.smoother == DGMG_SMOOTHER_EA) {
      int rc = k_sweep<T>(h, l, -1, u, f, r, u_zero && s == 0);
      if (rc) return rc;
    } else {
      for (int d = 0; d < h->lv[l].dim; ++d) {
        int rc = k_sweep<T>(h, l, d, u, f, r, u_zero && s == 0 && d == 0);
        if (rc) return rc;
      }
    }
  }
  return DGMG_OK;
}

template <class T>
int k_transfer(dgmg_handle* h, int l, bool restr, const T* in, T* out) {
  const LevelDev<T>& L = LD<T>(h, l);
  T* tmp = (T*)h->patch;
  if (L.se) {
    const LevelDev<T>& Lc = LD<T>(h, l - 1);
    int rc = L.dim == 3 ? Kern<T, 3>::se_transfer(L, Lc, restr, in, out, tmp, h->stream)
                        : Kern<T, 2>::se_transfer(L, Lc, restr, in, out, tmp, h->stream);
    if (rc) return fail(h, DGMG_EUNSUPPORTED, "no continuous transfer kernel for this order pair");
    return check_hip(h, "transfer");
  }
  int rc = L.dim == 3 ? Kern<T, 3>::transfer(L, restr, in, out, tmp, h->stream)
                      : Kern<T, 2>::transfer(L, restr, in, out, tmp, h->stream);
  if (rc) return fail(h, DGMG_EUNSUPPORTED, "no transfer kernel for this order pair");
  return check_hip(h, "transfer");
}

// f_{l-1} = restriction of (f_l - A_l u_l): one fused launch where it is built
// (the fine residual then never leaves LDS), else the residual into r_scratch
// and the transfer.  Both give the same values.
template <class T>
int k_residual_restrict(dgmg_handle* h, int l, const T* u, const T* f, T* r_scratch, T* fc) {
  const LevelDev<T>& L = LD<T>(h, l);
  T* scratch = (T*)h->patch;
  int rc = -4;
  if (h->fuse_restrict && !L.se)
    rc = L.dim == 3 ? Kern<T, 3>::apply(L, 3, u, f, fc, scratch, nullptr, nullptr, h->stream)
                    : Kern<T, 2>::apply(L, 3, u, f, fc, scratch, nullptr, nullptr, h->stream);
  if (rc == 0) return check_hip(h, "residual restriction");
  rc = k_apply<T>(h, l, 1, u, f, r_scratch, nullptr, nullptr);
  if (rc) return rc;
  return k_transfer<T>(h, l, true, r_scratch, fc);
}


// sum of a (n doubles) into *out, using c_a as a vector of ones
void k_mean_sub(dgmg_handle* h, double* a, int64_t n) {
  k_fill_v<double>(h, h->c_a, n, 1.0);
  hipLaunchKernelGGL(k_dot, dim3(RED_BLOCKS), dim3(VEC_THREADS), 0, h->stream, a, h->c_a, n, h->part, h->active);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(VEC_THREADS), 0, h->stream, h->part, RED_BLOCKS, h->scal + 41, h->active);
  hipLaunchKernelGGL(k_sub_scalar, dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, a, h->scal + 41,
                     1.0 / (double)n, n, h->active);
}

// u0 = A0^+ f0 (double vectors) by global fast diagonalisation.
int coarse_fdm(dgmg_handle* h, const double* f0, double* u0) {
  const LevelHost& l0 = h->lv[0];
  const int64_t n = l0.n_dof;
  const unsigned nb = (unsigned)((n + VEC_THREADS - 1) / VEC_THREADS);
  const int dim = l0.dim;
  const double* src = f0;
  bool periodic_all = true;
  for (int d = 0; d < dim; ++d) periodic_all = periodic_all && l0.dir[d].periodic;
  if (periodic_all) {  // make f0 orthogonal to the constants (Euclidean mean)
    hipLaunchKernelGGL(k_copy, dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, f0, h->c_f, n, h->active);
    k_mean_sub(h, h->c_f, n);
    src = h->c_f;
  }
  double* bufs[2] = {h->c_a, h->c_b};
  const double* in = src;
  int k = 0;
  for (int d = 0; d < dim; ++d) {
    double* out = bufs[k];
    if (h->cdev.se) {
      if (d == dim - 1)
        hipLaunchKernelGGL((k_coarse_pass_lat<true, true>), dim3(nb), dim3(VEC_THREADS), 0, h->stream, h->cdev, d, in, out, n, h->active);
      else
        hipLaunchKernelGGL((k_coarse_pass_lat<true, false>), dim3(nb), dim3(VEC_THREADS), 0, h->stream, h->cdev, d, in, out, n, h->active);
    } else if (d == dim - 1)
      hipLaunchKernelGGL((k_coarse_pass<true, true>), dim3(nb), dim3(VEC_THREADS), 0, h->stream, h->cdev, d, in, out, n, h->active);
    else
      hipLaunchKernelGGL((k_coarse_pass<true, false>), dim3(nb), dim3(VEC_THREADS), 0, h->stream, h->cdev, d, in, out, n, h->active);
    in = out;
    k ^= 1;
  }
  for (int d = dim - 1; d >= 0; --d) {
    double* out = d == 0 ? u0 : bufs[k];
    if (h->cdev.se)
      hipLaunchKernelGGL((k_coarse_pass_lat<false, false>), dim3(nb), dim3(VEC_THREADS), 0, h->stream, h->cdev, d, in, out, n, h->active);
    else
      hipLaunchKernelGGL((k_coarse_pass<false, false>), dim3(nb), dim3(VEC_THREADS), 0, h->stream, h->cdev, d, in, out, n, h->active);
    in = out;
    k ^= 1;
  }
  if (periodic_all) k_mean_sub(h, u0, n);  // mean-free (minimum-norm) representative
  return check_hip(h, "coarse solve");
}

template <class T>
int k_coarse(dgmg_handle* h, const T* f0, T* u0);
template <>
int k_coarse<double>(dgmg_handle* h, const double* f0, double* u0) { return coarse_fdm(h, f0, u0); }
template <>
int k_coarse<float>(dgmg_handle* h, const float* f0, float* u0) {
  const int64_t n = h->lv[0].n_dof;
  // FP64 copies: input in the level-0 residual buffer (sized for doubles), result
  // in the patch buffer (c_a, c_b and c_f are used by coarse_fdm)
  double* tmp_in = (double*)h->buf[0].r;
  double* res = (double*)h->patch;
  hipLaunchKernelGGL((k_convert<float, double>), dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, f0, tmp_in, n, h->active);
  int rc = coarse_fdm(h, tmp_in, res);
  if (rc) return rc;
  hipLaunchKernelGGL((k_convert<double, float>), dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, res, u0, n, h->active);
  return check_hip(h, "coarse convert");
}

// z = MultigridCycle(0, r) on multigrid-precision vectors (Alg. 1).
template <class T>
int k_vcycle(dgmg_handle* h, const T* r, T* z) {
  const int L = (int)h->lv.size() - 1;
  std::vector<T*> u(L + 1), f(L + 1);
  for (int l = 0; l <= L; ++l) {
    u[l] = (T*)h->buf[l].u;
    f[l] = (T*)h->buf[l].f;
  }
  u[L] = z;
  f[L] = const_cast<T*>(r);
  const bool var = h->opts.vcycle == DGMG_VCYCLE_VARIABLE;
  auto ns = [&](int l, int which) {
    const int base = which == 0 ? h->opts.ns_pre : h->opts.ns_post;
    return var ? base << (L - l) : base;
  };
  for (int l = L; l >= 1; --l) {
    // with pre-smoothing its first sweep assigns u (u_zero); without, u starts from zero
    const bool pre = ns(l, 0) > 0;
    if (!pre) k_fill_v<T>(h, u[l], h->lv[l].n_dof);
    T* rl = (T*)h->buf[l].r;
    int rc = k_smooth<T>(h, l, u[l], f[l], ns(l, 0), rl, pre);
    if (rc) return rc;
    rc = k_residual_restrict<T>(h, l, u[l], f[l], rl, f[l - 1]);
    if (rc) return rc;
  }
  int rc = k_coarse<T>(h, f[0], u[0]);
  if (rc) return rc;
  for (int l = 1; l <= L; ++l) {
    rc = k_transfer<T>(h, l, false, u[l - 1], u[l]);
    if (rc) return rc;
    rc = k_smooth<T>(h, l, u[l], f[l], ns(l, 1), (T*)h->buf[l].r);
    if (rc) return rc;
  }
  return DGMG_OK;
}

// Preconditioner z = MG(r) on FP64 top-level vectors.
// widen = false (mixed precision only): the FP32 result stays in the top
// level's u buffer and z is not written (the caller widens it itself).
// narrow = false: the FP32 copy of r is already in the top level's f buffer.
int precond(dgmg_handle* h, const double* r, double* z, bool widen = true, bool narrow = true) {
  const int L = (int)h->lv.size() - 1;
  const int64_t n = h->lv[L].n_dof;
  if (!mixed(h)) return k_vcycle<double>(h, r, z);
  float* rf = (float*)h->buf[L].f;
  float* zf = (float*)h->buf[L].u;
  if (narrow)
    hipLaunchKernelGGL((k_convert<double, float>), dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, r, rf, n, h->active);
  int rc = k_vcycle<float>(h, rf, zf);
  if (rc) return rc;
  if (widen)
    hipLaunchKernelGGL((k_convert<float, double>), dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, zf, z, n, h->active);
  return check_hip(h, "precond convert");
}

// ---------------------------------------------------------------- MGCG phases (Alg. 2)
// Fixed device scalar slots so that a phase can be captured once and replayed.
enum { S_DELTA = 0, S_BETA = 1, S_PQ = 2, S_RR = 3, S_ZDR = 4, S_ZR = 5, S_ROW = 6, S_RTRUE = 7 };

double* rr_slot(dgmg_handle* h) { return h->rr_out ? h->rr_out : h->scal + S_RR; }

// r = g - A x; r_old = 0; r.r
int pcg_init_a(dgmg_handle* h, const double* rhs, const double* x) {
  const int L = (int)h->lv.size() - 1;
  const int64_t n = h->lv[L].n_dof;
  int rc = k_apply<double>(h, L, 1, x, rhs, h->pr, nullptr, nullptr);
  if (rc) return rc;
  // r_old enters with weight 0 until the first direction update (r_old = 0
  // initially); the first phase a writes it before any read
  k_fill_v<double>(h, h->scal + S_ROW, 1);
  hipLaunchKernelGGL(k_dot, dim3(RED_BLOCKS), dim3(VEC_THREADS), 0, h->stream, h->pr, h->pr, n, h->part, h->active);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(VEC_THREADS), 0, h->stream, h->part, RED_BLOCKS, rr_slot(h), h->active);
  return check_hip(h, "pcg init");
}

// p = MG(r); delta = p.r
int pcg_init_b(dgmg_handle* h) {
  const int L = (int)h->lv.size() - 1;
  const int64_t n = h->lv[L].n_dof;
  int rc = precond(h, h->pr, h->pp);
  if (rc) return rc;
  hipLaunchKernelGGL(k_dot, dim3(RED_BLOCKS), dim3(VEC_THREADS), 0, h->stream, h->pp, h->pr, n, h->part, h->active);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(VEC_THREADS), 0, h->stream, h->part, RED_BLOCKS, h->scal + S_DELTA, h->active);
  return check_hip(h, "pcg init");
}

// q = A p; alpha = delta / p.q; x += alpha p; r_old = r; r -= alpha q; r.r
int pcg_phase_a_tail(dgmg_handle* h, double* x, int nb);
int pcg_phase_a(dgmg_handle* h, double* x) {
  const int L = (int)h->lv.size() - 1;
  int nb = 0;
  int rc = k_apply<double>(h, L, 2, h->pp, nullptr, h->pq, h->part, &nb);
  if (rc) return rc;
  return pcg_phase_a_tail(h, x, nb);
}

// Phase a after q = A p (nb partial sums of p.q in part)
int pcg_phase_a_tail(dgmg_handle* h, double* x, int nb) {
  const int L = (int)h->lv.size() - 1;
  const int64_t n = h->lv[L].n_dof;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(VEC_THREADS), 0, h->stream, h->part, nb, h->scal + S_PQ, h->active);
  float* rf = mixed(h) ? (float*)h->buf[L].f : nullptr;  // the next V-cycle's FP32 input
  hipLaunchKernelGGL(k_update_xr, dim3(RED_BLOCKS), dim3(VEC_THREADS), 0, h->stream, x, h->pr, h->pro, h->pp, h->pq,
                     h->scal + S_DELTA, h->scal + S_PQ, n, h->part2, rf, h->active);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(VEC_THREADS), 0, h->stream, h->part2, RED_BLOCKS, rr_slot(h), h->active);
  return check_hip(h, "pcg phase a");
}

// z = MG(r); beta = z.(r - r_old) / delta; p = z + beta p; delta = z.r
int pcg_phase_b_tail(dgmg_handle* h);
int pcg_phase_b(dgmg_handle* h) {
  const int L = (int)h->lv.size() - 1;
  const int64_t n = h->lv[L].n_dof;
  // mixed precision: the dot products and the direction update read the FP32
  // V-cycle output and widen it (no FP64 z); r's FP32 copy was written by
  // phase a's update
  const bool mx = mixed(h);
  int rc = precond(h, h->pr, h->pz, !mx, !mx);
  if (rc) return rc;
  return pcg_phase_b_tail(h);
}

// Phase b after the V-cycle
int pcg_phase_b_tail(dgmg_handle* h) {
  const int L = (int)h->lv.size() - 1;
  const int64_t n = h->lv[L].n_dof;
  const bool mx = mixed(h);
  const float* zf = (const float*)h->buf[L].u;
  if (mx)
    hipLaunchKernelGGL((k_dot_zr<float>), dim3(RED_BLOCKS), dim3(VEC_THREADS), 0, h->stream, zf, h->pr, h->pro,
                       h->scal + S_ROW, n, h->part, h->part2, h->active);
  else
    hipLaunchKernelGGL((k_dot_zr<double>), dim3(RED_BLOCKS), dim3(VEC_THREADS), 0, h->stream, h->pz, h->pr, h->pro,
                       h->scal + S_ROW, n, h->part, h->part2, h->active);
  hipLaunchKernelGGL(k_finalize_beta, dim3(1), dim3(VEC_THREADS), 0, h->stream, h->part, h->part2, RED_BLOCKS,
                     h->scal, h->active);
  if (mx)
    hipLaunchKernelGGL((k_update_p<float>), dim3(RED_BLOCKS), dim3(VEC_THREADS), 0, h->stream, h->pp, zf,
                       h->scal + S_BETA, n, h->active);
  else
    hipLaunchKernelGGL((k_update_p<double>), dim3(RED_BLOCKS), dim3(VEC_THREADS), 0, h->stream, h->pp,
                       (const double*)h->pz, h->scal + S_BETA, n, h->active);
  return check_hip(h, "pcg phase b");
}

// Record `fn` into a graph.  The capture runs on a private non-blocking stream
// (the caller's stream may be the legacy default stream, which cannot be
// captured); the graph is later launched on the caller's stream.
template <class F>
int capture(dgmg_handle* h, hipGraph_t* g, F fn) {
  if (!h->cap_stream) {
    hipError_t e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(h, DGMG_EHIP, std::string("capture stream: ") + hipGetErrorString(e));
  }
  const bool t = h->timing;
  hipStream_t user = h->stream;
  h->timing = false;
  hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    h->timing = t;
    return fail(h, DGMG_EHIP, std::string("begin capture: ") + hipGetErrorString(e));
  }
  h->stream = h->cap_stream;
  int rc = fn();
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(h->cap_stream, &graph);
  h->stream = user;
  h->timing = t;
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return fail(h, DGMG_EHIP, std::string("end capture: ") + hipGetErrorString(e));
  *g = graph;
  return DGMG_OK;
}

void drop_graphs(dgmg_handle* h) {
  for (auto& g : h->gexec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  h->graph_x = nullptr;
}

int instantiate(dgmg_handle* h, hipGraph_t g, hipGraphExec_t* ex) {
  hipError_t e = hipGraphInstantiate(ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(h, DGMG_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
  return DGMG_OK;
}

int run_phase(dgmg_handle* h, int which, double* x) {
  if (!h->use_graphs) return which == 0 ? pcg_phase_a(h, x) : pcg_phase_b(h);
  if (which == 0 && h->gexec[0] && h->graph_x != x) {
    (void)hipGraphExecDestroy(h->gexec[0]);
    h->gexec[0] = nullptr;
  }
  if (!h->gexec[which]) {
    hipGraph_t g = nullptr;
    int rc = capture(h, &g, [&]() { return which == 0 ? pcg_phase_a(h, x) : pcg_phase_b(h); });
    if (rc) return rc;
    if ((rc = instantiate(h, g, &h->gexec[which]))) return rc;
    if (which == 0) h->graph_x = x;
  }
  hipError_t e = hipGraphLaunch(h->gexec[which], h->stream);
  if (e != hipSuccess) return fail(h, DGMG_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
  return DGMG_OK;
}

int read_scalar(dgmg_handle* h, const double* dev, double* out) {
  hipError_t e = hipMemcpyAsync(h->host_scal, dev, sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(h, DGMG_EHIP, std::string("scalar readback: ") + hipGetErrorString(e));
  *out = *h->host_scal;
  return DGMG_OK;
}

// Exit confirmation of Alg. 2: r = g - A x (FP64) and its norm.  The recursive
// residual of the PCG update and the true one drift apart by rounding; the
// solve stops only when the true residual meets the tolerance.  r overwrites
// the recursive residual, so when the check fails the iteration continues from
// the true residual (residual replacement); in mixed precision its FP32 copy,
// the next V-cycle's input, is refreshed as well.
int true_residual(dgmg_handle* h, const double* rhs, const double* x, double* norm) {
  const int L = (int)h->lv.size() - 1;
  const int64_t n = h->lv[L].n_dof;
  int rc = k_apply<double>(h, L, 1, x, rhs, h->pr, nullptr, nullptr);
  if (rc) return rc;
  hipLaunchKernelGGL(k_dot, dim3(RED_BLOCKS), dim3(VEC_THREADS), 0, h->stream, h->pr, h->pr, n, h->part, h->active);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(VEC_THREADS), 0, h->stream, h->part, RED_BLOCKS, h->scal + S_RTRUE,
                     h->active);
  if (mixed(h))
    hipLaunchKernelGGL((k_convert<double, float>), dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, h->pr,
                       (float*)h->buf[L].f, n, h->active);
  if ((rc = check_hip(h, "true residual"))) return rc;
  double rr;
  if ((rc = read_scalar(h, h->scal + S_RTRUE, &rr))) return rc;
  *norm = std::sqrt(rr);
  return DGMG_OK;
}

int need_bound(dgmg_handle* h) {
  if (!h) return DGMG_EINVAL;
  if (!h->bound) return fail(h, DGMG_ENOMEM, "workspace not bound");
  return DGMG_OK;
}

int check_level(dgmg_handle* h, int level, int minl = 0) {
  if (level < minl || level >= (int)h->lv.size()) return fail(h, DGMG_EINVAL, "level out of range");
  return DGMG_OK;
}

int validate_setup(const dgmg_grid* g, const dgmg_opts* o, SetupParams& sp) {
  if (!g || !o) return fail(nullptr, DGMG_EINVAL, "null argument");
  if (g->dim != 2 && g->dim != 3) return fail(nullptr, DGMG_EINVAL, "dim must be 2 or 3");
  if (o->P < 1 || o->P > 32) return fail(nullptr, DGMG_EINVAL, "P must be in 1 .. 32");
  // compiled kernels for P_l in {1, 2, 3, 4, 6, 8, 12, 16, 32}; other orders run
  // the run-time kernels, whose 3D tiles fit the LDS up to P = 17
  const int okP[] = {1, 2, 3, 4, 6, 8, 12, 16, 32};
  const bool compiled = std::find(std::begin(okP), std::end(okP), o->P) != std::end(okP);
  if (g->dim == 3 && o->P > 17 && o->P != 32)
    return fail(nullptr, DGMG_EUNSUPPORTED, "3D orders 18 .. 31 are not built (their patch tiles exceed the LDS)");
  if (o->disc == DGMG_DISC_SE && !compiled)
    return fail(nullptr, DGMG_EUNSUPPORTED, "the continuous counterpart needs P in 1, 2, 3, 4, 6, 8, 12, 16, 32");
  if (!(o->mu_star > 0) || !std::isfinite(o->mu_star)) return fail(nullptr, DGMG_EINVAL, "mu_star must be > 0");
  if (o->flux != DGMG_FLUX_IP && o->flux != DGMG_FLUX_LDG) return fail(nullptr, DGMG_EINVAL, "bad flux");
  if (o->smoother < DGMG_SMOOTHER_EA || o->smoother > DGMG_SMOOTHER_FM) return fail(nullptr, DGMG_EINVAL, "bad smoother");
  if (o->order != DGMG_ORDER_LEX && o->order != DGMG_ORDER_COLOUR) return fail(nullptr, DGMG_EINVAL, "bad order");
  const bool mult = o->smoother == DGMG_SMOOTHER_EM || o->smoother == DGMG_SMOOTHER_FM;
  if (o->weighting < 0 || o->weighting > 3) return fail(nullptr, DGMG_EINVAL, "bad weighting");
  if (o->vcycle != DGMG_VCYCLE_CLASSICAL && o->vcycle != DGMG_VCYCLE_VARIABLE) return fail(nullptr, DGMG_EINVAL, "bad vcycle");
  if (o->precision != DGMG_PREC_FP64 && o->precision != DGMG_PREC_MIXED) return fail(nullptr, DGMG_EINVAL, "bad precision");
  if (o->ns_pre < 0 || o->ns_post < 0 || o->max_iter < 0) return fail(nullptr, DGMG_EINVAL, "negative count");
  if (o->overlap < -2) return fail(nullptr, DGMG_EINVAL, "bad overlap");
  if (o->disc != DGMG_DISC_DG && o->disc != DGMG_DISC_SE) return fail(nullptr, DGMG_EINVAL, "bad discretisation");
  if (o->disc == DGMG_DISC_SE) {
    if (o->smoother != DGMG_SMOOTHER_EA)
      return fail(nullptr, DGMG_EUNSUPPORTED, "the continuous counterpart uses the element-centred additive smoother");
    if (g->dim == 3 && o->P > 16)
      return fail(nullptr, DGMG_EUNSUPPORTED, "continuous 3D levels need P <= 16 (element tiles in LDS)");
  }
  sp = SetupParams();
  sp.dim = g->dim;
  for (int d = 0; d < g->dim; ++d) {
    if (g->n_elem[d] < 1 || !g->dx[d]) return fail(nullptr, DGMG_EINVAL, "n_elem < 1 or dx missing");
    if (g->periodic[d] && g->n_elem[d] < 3) return fail(nullptr, DGMG_EINVAL, "periodic direction needs >= 3 elements");
    sp.n[d] = g->n_elem[d];
    sp.periodic[d] = g->periodic[d] != 0;
    sp.dx[d].assign(g->dx[d], g->dx[d] + g->n_elem[d]);
    for (double v : sp.dx[d])
      if (!(v > 0) || !std::isfinite(v)) return fail(nullptr, DGMG_EINVAL, "dx must be finite and > 0");
    if (o->flux == DGMG_FLUX_LDG && !(std::fabs(o->beta[d]) <= 1.0)) return fail(nullptr, DGMG_EINVAL, "|beta| must be <= 1");
  }
  int64_t ne = 1;
  for (int d = 0; d < g->dim; ++d) ne *= g->n_elem[d];
  if (ne * (int64_t)std::pow(o->P + 1, g->dim) > (int64_t)INT32_MAX)
    return fail(nullptr, DGMG_EINVAL, "problem too large (at most 2^31 - 1 unknowns)");
  sp.P = o->P;
  sp.flux = o->flux;
  for (int d = 0; d < 3; ++d) sp.beta[d] = o->beta[d];
  sp.mu_star = o->mu_star;
  sp.smoother = o->smoother;
  sp.overlap = o->overlap;
  sp.disc = o->disc;
  // multiplicative Schwarz adds its corrections unweighted: unit weight tables
  sp.weighting = mult ? DGMG_WEIGHT_NONE : o->weighting;
  return DGMG_OK;
}

// Time the patch-solve block shapes of every sweep and keep the fastest.
template <class T>
int autotune_t(dgmg_handle* h) {
  const int nl = (int)h->lv.size();
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  int rc = DGMG_OK;
  for (int l = 1; l < nl && !rc; ++l) {
    T* r = (T*)h->buf[l].r;
    k_fill_v<T>(h, r, h->lv[l].n_dof);
    const int nkinds = ec_smoother(h) ? 1 : h->lv[l].dim;
    for (int q = 0; q < nkinds && !rc; ++q) {
      const int nd = ec_smoother(h) ? -1 : q;
      const int kind = nd < 0 ? 3 : nd;
      float best = 1e30f;
      int bw = 0;
      for (int w : {1, 2, 4, 8}) {
        if ((rc = k_fdm<T>(h, l, nd, r, w))) break;
        (void)hipEventRecord(e0, h->stream);
        for (int rep = 0; rep < 3; ++rep)
          if ((rc = k_fdm<T>(h, l, nd, r, w))) break;
        (void)hipEventRecord(e1, h->stream);
        if (rc) break;
        hipError_t e = hipEventSynchronize(e1);
        if (e != hipSuccess) {
          rc = fail(h, DGMG_EHIP, std::string("autotune: ") + hipGetErrorString(e));
          break;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
          best = ms;
          bw = w;
        }
      }
      h->waves[l][kind] = bw;
      h->tune_ms[l][kind] = best / 3.0f;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!rc) rc = check_hip(h, "autotune");
  drop_graphs(h);
  return rc;
}

int bind_batch_member(dgmg_handle* h, char* dev, hipStream_t s, const int* flag, double* rr) {
  h->active = flag;
  h->rr_out = rr;
  return dgmg_bind_workspace(h, dev, h->ws_need, s);
}

}  // namespace

// =================================================================== C ABI
extern "C" {

int dgmg_opts_default(dgmg_opts* o) {
  if (!o) return DGMG_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->P = 4;
  o->flux = DGMG_FLUX_IP;
  o->mu_star = 1.0;
  o->smoother = DGMG_SMOOTHER_FA;
  o->overlap = DGMG_OVERLAP_LEVEL;
  o->weighting = DGMG_WEIGHT_QUINTIC;
  o->vcycle = DGMG_VCYCLE_CLASSICAL;
  o->ns_pre = 1;
  o->ns_post = 1;
  o->precision = DGMG_PREC_FP64;
  o->max_iter = 100;
  return DGMG_OK;
}

int dgmg_setup(const dgmg_grid* g, const dgmg_opts* o, dgmg_handle** out) {
  if (!out) return fail(nullptr, DGMG_EINVAL, "null argument");
  *out = nullptr;
  SetupParams sp;
  int rc = validate_setup(g, o, sp);
  if (rc) return rc;
  dgmg_handle* h = new dgmg_handle();
  h->fuse_restrict = std::getenv("DGMG_NO_FUSED_RESTRICTION") == nullptr;
  h->sp = sp;
  h->opts = *o;
  std::string e = build_levels(sp, h->lv);
  if (!e.empty()) {
    delete h;
    return fail(nullptr, DGMG_EINVAL, e);
  }
  if ((int)h->lv.size() > MAXL) {
    delete h;
    return fail(nullptr, DGMG_EUNSUPPORTED, "too many levels");
  }
  for (size_t l = 1; l < h->lv.size(); ++l) {  // kernels must exist for every smoothing level
    const LevelHost& lv = h->lv[l];
    const int NL = lv.NP + 2 * lv.NO;
    const int NA = (o->smoother == DGMG_SMOOTHER_EA || o->smoother == DGMG_SMOOTHER_EM) ? NL : 2 * lv.P;
    const bool ok = g->dim == 3 ? Kern<double, 3>::fdm_supported(NA, NL) : Kern<double, 2>::fdm_supported(NA, NL);
    if (!ok) {
      delete h;
      return fail(nullptr, DGMG_EUNSUPPORTED,
                  "no patch kernel for P_l=" + std::to_string(lv.P) + " N_O=" + std::to_string(lv.NO));
    }
    // the multiplicative launches take subsets of the patches: only the tiles that fit in LDS
    if (multiplicative(h) && g->dim == 3 && !Kern<double, 3>::fdm_in_lds(NA, NL)) {
      delete h;
      return fail(nullptr, DGMG_EUNSUPPORTED,
                  "multiplicative smoothers: the patch tile of P_l=" + std::to_string(lv.P) +
                      " exceeds LDS (its large-tile solve takes whole partitions only)");
    }
  }
  if (multiplicative(h))
    for (size_t l = 1; l < h->lv.size(); ++l) {
      if (ec_smoother(h)) h->mcls[l][3] = mult_classes(h->lv[l], -1, o->order);
      else
        for (int d = 0; d < h->lv[l].dim; ++d) h->mcls[l][d] = mult_classes(h->lv[l], d, o->order);
    }
  layout(h, nullptr, nullptr);
  *out = h;
  return DGMG_OK;
}

int dgmg_workspace_bytes(const dgmg_handle* h, size_t* bytes) {
  if (!h || !bytes) return DGMG_EINVAL;
  *bytes = h->ws_need;
  return DGMG_OK;
}

int dgmg_bind_workspace(dgmg_handle* h, void* dev, size_t bytes, void* stream) {
  if (!h || !dev) return DGMG_EINVAL;
  if (bytes < h->ws_need) return fail(h, DGMG_ENOMEM, "workspace too small");
  if (((uintptr_t)dev) & 255) return fail(h, DGMG_EINVAL, "workspace must be 256-byte aligned");
  drop_graphs(h);
  h->stream = (hipStream_t)stream;
  h->ws = (char*)dev;
  h->ws_bytes = bytes;
  Upload up;
  layout(h, h->ws, &up);
  for (auto& u : up) {
    hipError_t e = hipMemcpyAsync(u.first, u.second.data(), u.second.size(), hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return fail(h, DGMG_EHIP, std::string("table upload: ") + hipGetErrorString(e));
  }
  if (!h->host_scal) {
    hipError_t e = hipHostMalloc((void**)&h->host_scal, 64 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) return fail(h, DGMG_EHIP, std::string("pinned alloc: ") + hipGetErrorString(e));
  }
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(h, DGMG_EHIP, std::string("bind sync: ") + hipGetErrorString(e));
  h->bound = true;
  return DGMG_OK;
}

int dgmg_set_stream(dgmg_handle* h, void* stream) {
  if (!h) return DGMG_EINVAL;
  if (h->stream != (hipStream_t)stream) drop_graphs(h);
  h->stream = (hipStream_t)stream;
  return DGMG_OK;
}

int dgmg_use_graphs(dgmg_handle* h, int enable) {
  if (!h) return DGMG_EINVAL;
  drop_graphs(h);
  h->use_graphs = enable != 0;
  return DGMG_OK;
}

int dgmg_num_levels(const dgmg_handle* h) { return h ? (int)h->lv.size() : DGMG_EINVAL; }

int dgmg_level_info(const dgmg_handle* h, int level, int* P, int* n_o, int64_t* n_dof) {
  if (!h || level < 0 || level >= (int)h->lv.size()) return DGMG_EINVAL;
  if (P) *P = h->lv[level].P;
  if (n_o) *n_o = h->lv[level].NO;
  if (n_dof) *n_dof = h->lv[level].n_dof;
  return DGMG_OK;
}

int dgmg_node_coords(const dgmg_handle* h, int level, int d, double* x) {
  if (!h || !x || level < 0 || level >= (int)h->lv.size() || d < 0 || d >= h->sp.dim) return DGMG_EINVAL;
  const LevelHost& lv = h->lv[level];
  std::vector<double> eta, rho;
  gll_points(lv.P, eta, rho);
  if (lv.se) {  // stored lattice nodes of the direction
    const Dir1D& dd = lv.dir[d];
    const int shift = dd.periodic ? 0 : 1;
    double left = 0.0;
    for (int m = 0; m < dd.N; ++m) {
      for (int i = 0; i < lv.P; ++i) {
        const int s = m * lv.P + i - shift;
        if (s >= 0 && s < dd.nl) x[s] = left + 0.5 * (1.0 + eta[i]) * dd.dx[m];
      }
      left += dd.dx[m];
    }
    return DGMG_OK;
  }
  double left = 0.0;
  for (int m = 0; m < lv.dir[d].N; ++m) {
    const double hh = lv.dir[d].dx[m];
    for (int i = 0; i < lv.NP; ++i) x[m * lv.NP + i] = left + 0.5 * (1.0 + eta[i]) * hh;
    left += hh;
  }
  return DGMG_OK;
}

int dgmg_apply(dgmg_handle* h, int level, const void* x, void* y, int dtype) {
  int rc = need_bound(h);
  if (rc || (rc = check_level(h, level))) return rc;
  if (!x || !y || x == y) return fail(h, DGMG_EINVAL, "x, y must be distinct device pointers");
  return dtype == DGMG_F64 ? k_apply<double>(h, level, 0, (const double*)x, nullptr, (double*)y, nullptr, nullptr)
                           : k_apply<float>(h, level, 0, (const float*)x, nullptr, (float*)y, nullptr, nullptr);
}

int dgmg_residual(dgmg_handle* h, int level, const void* f, const void* x, void* r, int dtype) {
  int rc = need_bound(h);
  if (rc || (rc = check_level(h, level))) return rc;
  if (!x || !r || !f || x == r) return fail(h, DGMG_EINVAL, "bad pointers");
  return dtype == DGMG_F64 ? k_apply<double>(h, level, 1, (const double*)x, (const double*)f, (double*)r, nullptr, nullptr)
                           : k_apply<float>(h, level, 1, (const float*)x, (const float*)f, (float*)r, nullptr, nullptr);
}

int dgmg_smooth(dgmg_handle* h, int level, void* u, const void* f, int nsteps, int dtype) {
  int rc = need_bound(h);
  if (rc || (rc = check_level(h, level, 1))) return rc;
  if (!u || !f || nsteps < 0) return fail(h, DGMG_EINVAL, "bad arguments");
  // residual scratch: the level buffer r and the patch buffer are sized for doubles
  if (dtype == DGMG_F64)
    return k_smooth<double>(h, level, (double*)u, (const double*)f, nsteps, (double*)h->buf[level].r);
  return k_smooth<float>(h, level, (float*)u, (const float*)f, nsteps, (float*)h->buf[level].r);
}

int dgmg_sweep(dgmg_handle* h, int level, void* u, const void* f, int normal, int dtype) {
  int rc = need_bound(h);
  if (rc || (rc = check_level(h, level, 1))) return rc;
  const LevelHost& lv = h->lv[level];
  if (!u || !f || normal < -1 || normal >= lv.dim) return fail(h, DGMG_EINVAL, "bad arguments");
  if (lv.se && normal != -1) return fail(h, DGMG_EINVAL, "continuous levels have element-centred subdomains only");
  int np[3], NA, NL;
  sweep_shape(lv, normal, np, NA, NL);
  const bool ok = lv.dim == 3 ? Kern<double, 3>::fdm_supported(NA, NL) : Kern<double, 2>::fdm_supported(NA, NL);
  if (!ok) return fail(h, DGMG_EUNSUPPORTED, "no patch kernel for this sweep");
  if (multiplicative(h) && (normal < 0) != ec_smoother(h))
    return fail(h, DGMG_EINVAL, "normal does not match the multiplicative smoother's subdomains");
  if (multiplicative(h)) {
    if (dtype == DGMG_F64)
      return k_msweep<double>(h, level, normal, (double*)u, (const double*)f, (double*)h->buf[level].r, false, false);
    return k_msweep<float>(h, level, normal, (float*)u, (const float*)f, (float*)h->buf[level].r, false, false);
  }
  if (dtype == DGMG_F64)
    return k_sweep<double>(h, level, normal, (double*)u, (const double*)f, (double*)h->buf[level].r);
  return k_sweep<float>(h, level, normal, (float*)u, (const float*)f, (float*)h->buf[level].r);
}

int dgmg_restrict(dgmg_handle* h, int level, const void* rf, void* fc, int dtype) {
  int rc = need_bound(h);
  if (rc || (rc = check_level(h, level, 1))) return rc;
  return dtype == DGMG_F64 ? k_transfer<double>(h, level, true, (const double*)rf, (double*)fc)
                           : k_transfer<float>(h, level, true, (const float*)rf, (float*)fc);
}

int dgmg_prolong(dgmg_handle* h, int level, const void* uc, void* uf, int dtype) {
  int rc = need_bound(h);
  if (rc || (rc = check_level(h, level, 1))) return rc;
  return dtype == DGMG_F64 ? k_transfer<double>(h, level, false, (const double*)uc, (double*)uf)
                           : k_transfer<float>(h, level, false, (const float*)uc, (float*)uf);
}

int dgmg_coarse_solve(dgmg_handle* h, const void* f0, void* u0, int dtype) {
  int rc = need_bound(h);
  if (rc) return rc;
  return dtype == DGMG_F64 ? k_coarse<double>(h, (const double*)f0, (double*)u0)
                           : k_coarse<float>(h, (const float*)f0, (float*)u0);
}

int dgmg_vcycle(dgmg_handle* h, const void* r, void* z, int dtype) {
  int rc = need_bound(h);
  if (rc) return rc;
  if ((dtype == DGMG_F32) != mixed(h)) return fail(h, DGMG_EINVAL, "dtype must match the handle precision");
  return dtype == DGMG_F64 ? k_vcycle<double>(h, (const double*)r, (double*)z)
                           : k_vcycle<float>(h, (const float*)r, (float*)z);
}

int dgmg_mass(dgmg_handle* h, const double* f, double* g) {
  int rc = need_bound(h);
  if (rc) return rc;
  const LevelDev<double>& L = h->Ld.back();
  if (L.se) hipLaunchKernelGGL(k_mass_se, dim3((unsigned)((L.n_dof + 255) / 256)), dim3(256), 0, h->stream, L, f, g);
  else hipLaunchKernelGGL(k_mass, dim3((unsigned)((L.n_dof + 255) / 256)), dim3(256), 0, h->stream, L, f, g);
  return check_hip(h, "mass");
}

// On a grid periodic in every direction A is singular (the constants span its
// null space): the system is consistent only for a right-hand side orthogonal
// to them.  Other grids pass at once.
static int check_rhs_consistent(dgmg_handle* h, const double* rhs) {
  const LevelHost& top = h->lv.back();
  bool periodic_all = true;
  for (int d = 0; d < top.dim; ++d) periodic_all = periodic_all && top.dir[d].periodic;
  if (!periodic_all) return DGMG_OK;
  hipLaunchKernelGGL(k_sum_abs, dim3(RED_BLOCKS), dim3(VEC_THREADS), 0, h->stream, rhs, top.n_dof, h->part,
                     h->part2, h->active);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(VEC_THREADS), 0, h->stream, h->part, RED_BLOCKS, h->scal + 42, h->active);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(VEC_THREADS), 0, h->stream, h->part2, RED_BLOCKS, h->scal + 43, h->active);
  double sum, asum;
  int rc;
  if ((rc = read_scalar(h, h->scal + 42, &sum)) || (rc = read_scalar(h, h->scal + 43, &asum))) return rc;
  if (!(std::fabs(sum) <= 1e-10 * asum))
    return fail(h, DGMG_EINVAL, "fully periodic grid: the right-hand side must sum to zero");
  return DGMG_OK;
}

int dgmg_solve(dgmg_handle* h, const double* rhs, double* x, double tol, dgmg_stats* st) {
  int rc = need_bound(h);
  if (rc) return rc;
  if (!rhs || !x || !(tol >= 0)) return fail(h, DGMG_EINVAL, "bad arguments");
  if (h->active) return fail(h, DGMG_EINVAL, "handle belongs to a batch");
  if (st) std::memset(st, 0, sizeof(*st));
  if ((rc = check_rhs_consistent(h, rhs))) return rc;
  if ((rc = pcg_init_a(h, rhs, x))) return rc;
  double rr;
  if ((rc = read_scalar(h, rr_slot(h), &rr))) return rc;
  const double r0 = std::sqrt(rr);
  if (!std::isfinite(r0)) return fail(h, DGMG_ENONFINITE, "initial residual is not finite");
  if (st) {
    st->r0 = r0;
    st->r_final = r0;
    st->history[0] = r0;
    st->converged = r0 == 0.0;
  }
  if (r0 == 0.0) return DGMG_OK;
  const double rmax = tol * r0;
  if ((rc = pcg_init_b(h))) return rc;
  double rn = r0;
  bool conv = false;
  for (int it = 1; it <= h->opts.max_iter; ++it) {
    if ((rc = run_phase(h, 0, x))) return rc;
    if ((rc = read_scalar(h, rr_slot(h), &rr))) return rc;
    rn = std::sqrt(rr);
    if (st) {
      st->iterations = it;
      st->r_final = rn;
      if (it < 256) st->history[it] = rn;
    }
    if (!std::isfinite(rn)) return fail(h, DGMG_ENONFINITE, "residual norm is not finite");
    if (rn <= rmax) {
      double rt;
      if ((rc = true_residual(h, rhs, x, &rt))) return rc;
      if (st) st->r_true = rt;
      if (rt <= rmax) {
        conv = true;
        break;
      }
      if (st) st->replacements++;
    }
    if ((rc = run_phase(h, 1, nullptr))) return rc;
  }
  if ((rc = check_hip(h, "pcg"))) return rc;
  if (st) {
    st->converged = conv;
    if (st->iterations > 0) st->rho = std::pow(rn / r0, 1.0 / st->iterations);
  }
  return conv ? DGMG_OK : DGMG_NOT_CONVERGED;
}

int dgmg_autotune(dgmg_handle* h) {
  int rc = need_bound(h);
  if (rc) return rc;
  return mixed(h) ? autotune_t<float>(h) : autotune_t<double>(h);
}

int dgmg_tune_get(const dgmg_handle* h, int level, int kind, int* waves, double* ms) {
  if (!h || level < 1 || level >= (int)h->lv.size() || kind < 0 || kind >= NKIND) return DGMG_EINVAL;
  if (waves) *waves = h->waves[level][kind];
  if (ms) *ms = h->tune_ms[level][kind];
  return DGMG_OK;
}

int dgmg_tune_set(dgmg_handle* h, int level, int kind, int waves) {
  if (!h || level < 1 || level >= (int)h->lv.size() || kind < 0 || kind >= NKIND || waves < 0 || waves > 8)
    return DGMG_EINVAL;
  h->waves[level][kind] = waves;
  drop_graphs(h);
  return DGMG_OK;
}

int dgmg_kernel_timing(dgmg_handle* h, int enable) {
  if (!h) return DGMG_EINVAL;
  if (enable < 0) return fail(h, DGMG_EINVAL, "kernel timing: negative stride");
  for (auto& e : h->ev) {
    h->ev_pool.push_back(e.first);
    h->ev_pool.push_back(e.second);
  }
  h->ev.clear();
  if (enable) {
    // events for a few hundred timed launches, created before any timed region
    while (h->ev_pool.size() < 1024) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) break;
      h->ev_pool.push_back(e);
    }
  } else {
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    h->ev_pool.clear();
  }
  h->ev_flops.clear();
  h->ev_bytes.clear();
  h->t_ms = h->t_flops = h->t_bytes = 0;
  h->t_launch = 0;
  h->timing = enable != 0;
  h->timing_stride = enable > 1 ? enable : 1;
  h->timing_count = 0;
  return DGMG_OK;
}

int dgmg_kernel_time(dgmg_handle* h, double* total_ms, int64_t* launches, double* flops, double* bytes) {
  if (!h) return DGMG_EINVAL;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(h, DGMG_EHIP, hipGetErrorString(e));
  for (size_t i = 0; i < h->ev.size(); ++i) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, h->ev[i].first, h->ev[i].second);
    h->t_ms += ms;
    h->t_flops += h->ev_flops[i];
    h->t_bytes += h->ev_bytes[i];
    h->t_launch += 1;
    h->ev_pool.push_back(h->ev[i].first);
    h->ev_pool.push_back(h->ev[i].second);
  }
  h->ev.clear();
  h->ev_flops.clear();
  h->ev_bytes.clear();
  if (total_ms) *total_ms = h->t_ms;
  if (launches) *launches = h->t_launch;
  if (flops) *flops = h->t_flops;
  if (bytes) *bytes = h->t_bytes;
  return DGMG_OK;
}

void dgmg_destroy(dgmg_handle* h) {
  if (!h) return;
  dgmg_kernel_timing(h, 0);
  drop_graphs(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->host_scal) (void)hipHostFree(h->host_scal);
  delete h;
}

const char* dgmg_last_error(const dgmg_handle* h) { return h ? h->err.c_str() : g_setup_error.c_str(); }

// ------------------------------------------------------------ learned face weights
}  // extern "C"

namespace {

// Upload the face-centred normal weights of every smoothing level (FP64 and
// FP32 tables): the fixed weights when theta is null, else the parametrised ones.
int upload_face_weights(dgmg_handle* h, const double* theta, const double* omega) {
  std::vector<std::vector<char>> keep;
  size_t off = 0;
  for (size_t l = 1; l < h->lv.size(); ++l) {
    const LevelHost& lv = h->lv[l];
    for (int d = 0; d < lv.dim; ++d) {
      const Dir1D& dd = lv.dir[d];
      std::vector<double> w;
      if (theta) fc_weights_param(lv, d, h->sp.weighting, theta + off, omega + off, w);
      else w = dd.w_fc;
      off += dd.nf;
      std::vector<char> b64(w.size() * sizeof(double)), b32(w.size() * sizeof(float));
      std::memcpy(b64.data(), w.data(), b64.size());
      float* f = reinterpret_cast<float*>(b32.data());
      for (size_t i = 0; i < w.size(); ++i) f[i] = (float)w[i];
      hipError_t e = hipMemcpyAsync((void*)h->Ld[l].dir[d].w_fc, b64.data(), b64.size(), hipMemcpyHostToDevice,
                                    h->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync((void*)h->Lf[l].dir[d].w_fc, b32.data(), b32.size(), hipMemcpyHostToDevice, h->stream);
      if (e != hipSuccess) return fail(h, DGMG_EHIP, std::string("weight upload: ") + hipGetErrorString(e));
      keep.push_back(std::move(b64));
      keep.push_back(std::move(b32));
    }
  }
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(h, DGMG_EHIP, std::string("weight upload sync: ") + hipGetErrorString(e));
  if (theta) {
    h->face_theta.assign(theta, theta + off);
    h->face_omega.assign(omega, omega + off);
  } else {
    h->face_theta.clear();
    h->face_omega.clear();
  }
  return DGMG_OK;
}

struct MlpWork {
  float *X, *Y, *hid;
  double *rhs, *x;
  size_t bytes;
};

MlpWork mlp_layout(const dgmg_handle* h, char* base) {
  const size_t nf = (size_t)face_count(h->lv), n = (size_t)h->lv.back().n_dof;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  MlpWork w{};
  size_t o = 0;
  w.X = (float*)(base + o);
  o += al(nf * DGMG_MLP_IN * sizeof(float));
  w.Y = (float*)(base + o);
  o += al(nf * DGMG_MLP_OUT * sizeof(float));
  w.hid = (float*)(base + o);
  o += al(nf * 2 * DGMG_MLP_HIDDEN * sizeof(float));
  w.rhs = (double*)(base + o);
  o += al(n * sizeof(double));
  w.x = (double*)(base + o);
  o += al(n * sizeof(double));
  w.bytes = o;
  return w;
}

// ||r_k|| / ||r_0|| after k PCG iterations from x = 0 on the probe right-hand side;
// +inf when the iteration breaks down (non-finite norms).
int probe_ratio(dgmg_handle* h, const MlpWork& w, int iters, double* ratio) {
  const int64_t n = h->lv.back().n_dof;
  hipLaunchKernelGGL(k_fill_hash, dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, w.rhs, n);
  k_fill_v<double>(h, w.x, n);
  const int save = h->opts.max_iter;
  h->opts.max_iter = iters;
  dgmg_stats st;
  int rc = dgmg_solve(h, w.rhs, w.x, 0.0, &st);
  h->opts.max_iter = save;
  if (rc == DGMG_ENONFINITE) {
    *ratio = INFINITY;
    return DGMG_OK;
  }
  if (rc < 0) return rc;
  *ratio = st.r0 > 0 ? st.r_final / st.r0 : 0.0;
  if (!std::isfinite(*ratio)) *ratio = INFINITY;
  return DGMG_OK;
}

}  // namespace

extern "C" {

int dgmg_face_count(const dgmg_handle* h) {
  if (!h) return DGMG_EINVAL;
  return face_count(h->lv);
}

int dgmg_face_features(const dgmg_handle* h, float* X) {
  if (!h || !X) return DGMG_EINVAL;
  std::vector<double> f;
  face_features(h->lv, f);
  for (size_t i = 0; i < f.size(); ++i) X[i] = (float)f[i];
  return DGMG_OK;
}

int dgmg_set_face_params(dgmg_handle* h, const double* theta, const double* omega) {
  int rc = need_bound(h);
  if (rc) return rc;
  if (h->opts.smoother != DGMG_SMOOTHER_FA)
    return fail(h, DGMG_EUNSUPPORTED, "face parameters need the face-centred smoother");
  if ((theta == nullptr) != (omega == nullptr)) return fail(h, DGMG_EINVAL, "theta and omega go together");
  if (theta) {
    const int n = face_count(h->lv);
    for (int i = 0; i < n; ++i)
      if (!(theta[i] > 0.0) || !(omega[i] > 0.0) || !std::isfinite(theta[i]) || !std::isfinite(omega[i]))
        return fail(h, DGMG_EINVAL, "theta and omega must be finite and > 0");
  }
  return upload_face_weights(h, theta, omega);
}

int dgmg_get_face_params(const dgmg_handle* h, double* theta, double* omega) {
  if (!h || !theta || !omega) return DGMG_EINVAL;
  const int n = face_count(h->lv);
  for (int i = 0; i < n; ++i) {
    theta[i] = h->face_theta.empty() ? 1.0 : h->face_theta[i];
    omega[i] = h->face_omega.empty() ? 1.0 : h->face_omega[i];
  }
  return h->face_theta.empty() ? 0 : 1;
}

int dgmg_mlp_work_bytes(const dgmg_handle* h, size_t* bytes) {
  if (!h || !bytes) return DGMG_EINVAL;
  *bytes = mlp_layout(h, nullptr).bytes;
  return DGMG_OK;
}

int dgmg_apply_mlp(dgmg_handle* h, const float* params, void* work, size_t bytes, int probe_iters,
                   double* ratios) {
  int rc = need_bound(h);
  if (rc) return rc;
  if (!params || !work || probe_iters < 1) return fail(h, DGMG_EINVAL, "bad arguments");
  if (h->active) return fail(h, DGMG_EINVAL, "handle belongs to a batch");
  if (h->opts.smoother != DGMG_SMOOTHER_FA)
    return fail(h, DGMG_EUNSUPPORTED, "learned weights need the face-centred smoother");
  if (((uintptr_t)work) & 255) return fail(h, DGMG_EINVAL, "work must be 256-byte aligned");
  const MlpWork w = mlp_layout(h, (char*)work);
  if (bytes < w.bytes) return fail(h, DGMG_ENOMEM, "MLP work buffer too small");
  const int nf = face_count(h->lv);
  // network outputs per face
  std::vector<double> feat;
  face_features(h->lv, feat);
  std::vector<float> X(feat.begin(), feat.end()), Y((size_t)nf * DGMG_MLP_OUT);
  hipError_t e = hipMemcpyAsync(w.X, X.data(), X.size() * sizeof(float), hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return fail(h, DGMG_EHIP, std::string("feature upload: ") + hipGetErrorString(e));
  if ((rc = dgmg_mlp_forward(params, w.X, nf, w.Y, w.hid, h->stream))) return fail(h, rc, "MLP forward");
  e = hipMemcpyAsync(Y.data(), w.Y, Y.size() * sizeof(float), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(h, DGMG_EHIP, std::string("MLP readback: ") + hipGetErrorString(e));
  std::vector<double> theta(nf), omega(nf);
  bool finite = true;
  for (int i = 0; i < nf; ++i) {
    const double y0 = Y[2 * i], y1 = Y[2 * i + 1];
    finite = finite && std::isfinite(y0) && std::isfinite(y1);
    theta[i] = DGMG_THETA_MIN + (DGMG_THETA_MAX - DGMG_THETA_MIN) / (1.0 + std::exp(-y0));
    omega[i] = DGMG_OMEGA_MIN + (DGMG_OMEGA_MAX - DGMG_OMEGA_MIN) / (1.0 + std::exp(-y1));
  }
  // probe: fixed weights first, then the learned ones
  double rf = 0, rl = INFINITY;
  if ((rc = upload_face_weights(h, nullptr, nullptr))) return rc;
  if ((rc = probe_ratio(h, w, probe_iters, &rf))) return rc;
  if (finite) {
    if ((rc = upload_face_weights(h, theta.data(), omega.data()))) return rc;
    if ((rc = probe_ratio(h, w, probe_iters, &rl))) return rc;
  }
  if (ratios) {
    ratios[0] = rl;
    ratios[1] = rf;
  }
  if (finite && rl <= rf) return DGMG_OK;
  if ((rc = upload_face_weights(h, nullptr, nullptr))) return rc;
  return DGMG_FELLBACK;
}

}  // extern "C"

// ------------------------------------------------------------------- batched execution plan
namespace {

// A batch whose grids share the multigrid precision, the smoothing counts and
// the V-cycle kind, with additive smoothers and no large (3D P = 32) levels,
// runs each MGCG phase as one list of launches over work lists (BatchList):
// every step of every grid's phase is keyed by its position (phase a: the
// top-level apply q = A p; phase b: the V-cycle, steps keyed by depth below the
// top level, smoothing step, sweep and sub-step), and the steps at one position
// that use the same kernel instance become one launch over all their grids,
// one argument descriptor per grid.  Each grid sees the same kernels on the
// same data in the same order as in its own solve (bitwise the same results).
// The PCG vector operations, fills and coarse solves stay per grid.
enum { BK_APPLY = 0, BK_FDM = 1, BK_COMB = 2, BK_XFER = 3, BK_FN = 4 };

struct BStep {
  std::vector<int> key;
  int kind = BK_FN, dim = 3, f32 = 0, t[4] = {0, 0, 0, 0};
  int grid = 0, nblk = 0;
  std::vector<char> args;
  std::function<int()> fn;
};

template <class A>
std::vector<char> arg_bytes(const A& a) {
  std::vector<char> v(sizeof(A));
  std::memcpy(v.data(), &a, sizeof(A));
  return v;
}

bool batch_plannable(const dgmg_batch* b) {
  const dgmg_handle* h0 = b->h[0];
  for (const dgmg_handle* h : b->h) {
    if (multiplicative(h)) return false;
    if (h->opts.precision != h0->opts.precision || h->opts.ns_pre != h0->opts.ns_pre ||
        h->opts.ns_post != h0->opts.ns_post || h->opts.vcycle != h0->opts.vcycle)
      return false;
    for (const LevelHost& lv : h->lv) {
      if (lv.dim == 3 && lv.NP == BIG_NP) return false;
      // run-time orders have no work-list launches
      if (!(lv.dim == 3 ? Kern<double, 3>::order_compiled(lv.NP) : Kern<double, 2>::order_compiled(lv.NP)))
        return false;
    }
  }
  return true;
}

// Levels with at least this many unknowns fill the GPU alone: their steps keep
// the single-grid launches (autotuned block shapes, arguments in scalar
// registers) and only the smaller levels share work-list launches.
constexpr int64_t SOLO_DOF = 1 << 20;

// Steps of one grid's V-cycle (as k_vcycle, k_smooth, k_sweep,
// k_residual_restrict and k_transfer issue them).
template <class T>
void vcycle_steps(dgmg_handle* h, int gi, const T* r_top, T* z_top, std::vector<BStep>& out) {
  const int L = (int)h->lv.size() - 1;
  const int f32 = sizeof(T) == 4;
  const bool var = h->opts.vcycle == DGMG_VCYCLE_VARIABLE;
  auto ns = [&](int l, int which) {
    const int base = which == 0 ? h->opts.ns_pre : h->opts.ns_post;
    return var ? base << (L - l) : base;
  };
  std::vector<T*> u(L + 1), f(L + 1);
  for (int l = 0; l <= L; ++l) {
    u[l] = (T*)h->buf[l].u;
    f[l] = (T*)h->buf[l].f;
  }
  u[L] = z_top;
  f[L] = const_cast<T*>(r_top);
  T* patch = (T*)h->patch;
  auto step = [&](std::vector<int> key, int kind, int dim, std::initializer_list<int> t, int nblk,
                  std::vector<char> args) {
    BStep st;
    st.key = std::move(key);
    st.kind = kind;
    st.dim = dim;
    st.f32 = f32;
    int k = 0;
    for (int v : t) st.t[k++] = v;
    st.grid = gi;
    st.nblk = nblk;
    st.args = std::move(args);
    out.push_back(std::move(st));
  };
  auto fnstep = [&](std::vector<int> key, std::function<int()> fn) {
    BStep st;
    st.key = std::move(key);
    st.kind = BK_FN;
    st.grid = gi;
    st.fn = std::move(fn);
    out.push_back(std::move(st));
  };
  auto blocks_apply = [&](const LevelDev<T>& Lv) {
    return Lv.dim == 3 ? Kern<T, 3>::apply_blocks_of(Lv.NP, Lv.n_elem) : Kern<T, 2>::apply_blocks_of(Lv.NP, Lv.n_elem);
  };
  auto apply_args = [&](const LevelDev<T>& Lv, const T* x, const T* fv, T* y) {
    ApplyArgs<T> a;
    a.L = Lv;
    a.x = x;
    a.f = fv;
    a.y = y;
    a.nblk = blocks_apply(Lv);
    return a;
  };
  // one smoothing call: steps s, sweeps i (EA: one, FA: one per direction);
  // keys {major, depthkey, s, i, sub-step}
  auto smooth = [&](int major, int depthkey, int l, int steps, bool u_zero) {
    const LevelDev<T>& Lv = LD<T>(h, l);
    const LevelHost& lv = h->lv[l];
    T* rl = (T*)h->buf[l].r;
    const int nsw = ec_smoother(h) ? 1 : lv.dim;
    const bool solo = lv.n_dof >= SOLO_DOF;
    for (int s = 0; s < steps; ++s)
      for (int i = 0; i < nsw; ++i) {
        const int nd = ec_smoother(h) ? -1 : i;
        const bool uz = u_zero && s == 0 && i == 0;
        if (solo) {
          T* ul = u[l];
          const T* fl = f[l];
          fnstep({major, depthkey, s, i, 0}, [h, l, nd, ul, fl, rl, uz]() { return k_sweep<T>(h, l, nd, ul, fl, rl, uz); });
          continue;
        }
        if (!uz) {
          ApplyArgs<T> a = apply_args(Lv, u[l], f[l], rl);
          step({major, depthkey, s, i, 0}, BK_APPLY, lv.dim, {lv.NP, 1}, a.nblk, arg_bytes(a));
        }
        int np[3], NA, NL;
        sweep_shape(lv, nd, np, NA, NL);
        FdmArgs<T> fa;
        fa.L = Lv;
        fa.r = uz ? f[l] : rl;
        fa.out = patch;
        fa.npx = np[0];
        fa.npy = np[1];
        fa.npz = np[2];
        step({major, depthkey, s, i, 1}, BK_FDM, lv.dim, {nd, NA, NL}, np[0] * np[1] * np[2], arg_bytes(fa));
        CombArgs<T> ca;
        ca.L = Lv;
        ca.buf = patch;
        ca.u = u[l];
        ca.nd = nd;
        ca.NA = NA;
        ca.NL = NL;
        ca.npx = np[0];
        ca.npy = np[1];
        ca.npz = np[2];
        ca.nblk = lv.dim == 3 ? Kern<T, 3>::combine_blocks_of(lv.NP, lv.n_elem)
                              : Kern<T, 2>::combine_blocks_of(lv.NP, lv.n_elem);
        ca.assign = uz ? 1 : 0;
        step({major, depthkey, s, i, 2}, BK_COMB, lv.dim, {lv.NP, combine_maxc(lv.NP, lv.NO)}, ca.nblk,
             arg_bytes(ca));
      }
  };
  auto xfer_args = [&](const LevelDev<T>& Lv, const T* in, T* o) {
    XferArgs<T> a;
    a.J = Lv.J;
    a.n_elem = Lv.n_elem;
    a.in = in;
    a.out = o;
    a.active = Lv.active;
    return a;
  };
  auto xfer_blocks = [&](const LevelDev<T>& Lv) {
    return Lv.dim == 3 ? Kern<T, 3>::xfer_blocks_of(Lv.NP, Lv.n_elem) : Kern<T, 2>::xfer_blocks_of(Lv.NP, Lv.n_elem);
  };
  for (int l = L; l >= 1; --l) {
    const int k = L - l;
    const bool pre = ns(l, 0) > 0;
    if (!pre) {
      T* ul = u[l];
      const int64_t n = h->lv[l].n_dof;
      fnstep({1, k, -1, 0, 0}, [h, ul, n]() {
        k_fill_v<T>(h, ul, n);
        return check_hip(h, "fill");
      });
    }
    smooth(1, k, l, ns(l, 0), pre);
    const LevelDev<T>& Lv = LD<T>(h, l);
    const LevelHost& lv = h->lv[l];
    // the fused form where built; the structure only depends on the orders
    // (J is null in a dry run before the workspace is bound)
    LevelDev<T> probe = Lv;
    if (!probe.J) probe.J = (const T*)&probe;
    const bool m3 = h->fuse_restrict &&
                    (lv.dim == 3 ? Kern<T, 3>::mode3_ok(probe) : Kern<T, 2>::mode3_ok(probe));
    T* rl = (T*)h->buf[l].r;
    if (lv.n_dof >= SOLO_DOF) {
      T* ul = u[l];
      const T* fl = f[l];
      T* fc = f[l - 1];
      fnstep({1, k, 1000, 0, 0}, [h, l, ul, fl, rl, fc]() { return k_residual_restrict<T>(h, l, ul, fl, rl, fc); });
    } else if (m3) {
      ApplyArgs<T> a = apply_args(Lv, u[l], f[l], f[l - 1]);
      step({1, k, 1000, 0, 0}, BK_APPLY, lv.dim, {lv.NP, 3}, a.nblk, arg_bytes(a));
    } else {
      ApplyArgs<T> a = apply_args(Lv, u[l], f[l], rl);
      step({1, k, 1000, 0, 0}, BK_APPLY, lv.dim, {lv.NP, 1}, a.nblk, arg_bytes(a));
      XferArgs<T> x = xfer_args(Lv, rl, f[l - 1]);
      step({1, k, 1000, 0, 1}, BK_XFER, lv.dim, {lv.NP, lv.NPc, 1}, xfer_blocks(Lv), arg_bytes(x));
    }
  }
  {
    T* f0 = f[0];
    T* u0 = u[0];
    fnstep({2}, [h, f0, u0]() { return k_coarse<T>(h, f0, u0); });
  }
  for (int l = 1; l <= L; ++l) {
    const int k = L - l;
    const LevelDev<T>& Lv = LD<T>(h, l);
    const LevelHost& lv = h->lv[l];
    if (lv.n_dof >= SOLO_DOF) {
      const T* uc = u[l - 1];
      T* ul = u[l];
      fnstep({3, -k, -1, 0, 0}, [h, l, uc, ul]() { return k_transfer<T>(h, l, false, uc, ul); });
    } else {
      XferArgs<T> x = xfer_args(Lv, u[l - 1], u[l]);
      step({3, -k, -1, 0, 0}, BK_XFER, lv.dim, {lv.NP, lv.NPc, 0}, xfer_blocks(Lv), arg_bytes(x));
    }
    smooth(3, -k, l, ns(l, 1), false);
  }
}

// Steps of both MGCG phases of every grid, merged into launches.  fill = false:
// a dry run (before the workspace is bound) that only sizes the descriptors.
int batch_plan(dgmg_batch* b, bool fill) {
  b->plan[0].clear();
  b->plan[1].clear();
  b->planned = batch_plannable(b);
  b->concurrent = false;
  for (const dgmg_handle* h : b->h) b->concurrent = b->concurrent || h->lv.back().n_dof >= SOLO_DOF;
  if (!b->planned) {
    b->plan_bytes = 0;
    return DGMG_OK;
  }
  std::vector<BStep> steps[2];
  const int n = (int)b->h.size();
  for (int gi = 0; gi < n; ++gi) {
    dgmg_handle* h = b->h[gi];
    const int L = (int)h->lv.size() - 1;
    // phase a: q = A p (top level, FP64), then the grid's own updates
    const LevelDev<double>& Lt = h->Ld[L];
    if (h->lv[L].n_dof >= SOLO_DOF) {
      BStep st;
      st.key = {0};
      st.grid = gi;
      const int64_t off = b->dof_off[gi];
      st.fn = [b, h, off]() { return pcg_phase_a(h, b->x_cur + off); };
      steps[0].push_back(std::move(st));
    } else {
    ApplyArgs<double> a;
    a.L = Lt;
    a.x = h->pp;
    a.y = h->pq;
    a.part = h->part;
    a.nblk = Lt.dim == 3 ? Kern<double, 3>::apply_blocks_of(Lt.NP, Lt.n_elem)
                         : Kern<double, 2>::apply_blocks_of(Lt.NP, Lt.n_elem);
    BStep st;
    st.key = {0};
    st.kind = BK_APPLY;
    st.dim = Lt.dim;
    st.f32 = 0;
    st.t[0] = Lt.NP;
    st.t[1] = 2;
    st.grid = gi;
    st.nblk = a.nblk;
    st.args = arg_bytes(a);
    steps[0].push_back(std::move(st));
    BStep tail;
    tail.key = {1};
    tail.grid = gi;
    const int nb = a.nblk;
    const int64_t off = b->dof_off[gi];
    tail.fn = [b, h, nb, off]() { return pcg_phase_a_tail(h, b->x_cur + off, nb); };
    steps[0].push_back(std::move(tail));
    }
    // phase b: the V-cycle (mixed: on the FP32 copies of r and z), then the direction update
    if (mixed(h)) vcycle_steps<float>(h, gi, (const float*)h->buf[L].f, (float*)h->buf[L].u, steps[1]);
    else vcycle_steps<double>(h, gi, h->pr, h->pz, steps[1]);
    BStep tb;
    tb.key = {9};
    tb.grid = gi;
    tb.fn = [h]() { return pcg_phase_b_tail(h); };
    steps[1].push_back(std::move(tb));
  }
  std::vector<char> host;
  auto alloc = [&](size_t bytes) {
    size_t o = (host.size() + 255) & ~size_t(255);
    host.resize(o + bytes);
    return o;
  };
  for (int ph = 0; ph < 2; ++ph) {
    auto& v = steps[ph];
    auto sig = [](const BStep& s) { return std::make_tuple(s.kind, s.dim, s.f32, s.t[0], s.t[1], s.t[2], s.t[3]); };
    std::stable_sort(v.begin(), v.end(), [&](const BStep& x, const BStep& y) {
      if (x.key != y.key) return x.key < y.key;
      if (sig(x) != sig(y)) return sig(x) < sig(y);
      return x.grid < y.grid;
    });
    for (size_t i = 0; i < v.size();) {
      size_t j = i + 1;
      while (j < v.size() && v[j].key == v[i].key && sig(v[j]) == sig(v[i])) ++j;
      dgmg_batch::Launch ln;
      ln.kind = v[i].kind;
      ln.key = v[i].key;
      ln.dim = v[i].dim;
      ln.f32 = v[i].f32;
      for (int k = 0; k < 4; ++k) ln.t[k] = v[i].t[k];
      ln.ng = (int)(j - i);
      if (ln.kind == BK_FN) {
        for (size_t k = i; k < j; ++k) {
          ln.fns.push_back(v[k].fn);
          ln.fn_grid.push_back(v[k].grid);
        }
      } else {
        const size_t asz = v[i].args.size();
        ln.desc_off = alloc(asz * ln.ng);
        for (size_t k = i; k < j; ++k) std::memcpy(host.data() + ln.desc_off + (k - i) * asz, v[k].args.data(), asz);
        ln.starts_off = alloc(sizeof(int) * (ln.ng + 1));
        int* st = (int*)(host.data() + ln.starts_off);
        st[0] = 0;
        for (size_t k = i; k < j; ++k) st[k - i + 1] = st[k - i] + v[k].nblk;
        ln.ntot = st[ln.ng];
      }
      b->plan[ph].push_back(std::move(ln));
      i = j;
    }
  }
  if (!fill) {
    b->plan_bytes = host.size() + 256;
    return DGMG_OK;
  }
  if (host.size() > b->plan_bytes) return DGMG_EINVAL;  // the dry run sized the region
  hipError_t e = hipMemcpyAsync(b->ws + b->plan_off, host.data(), host.size(), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  return e == hipSuccess ? DGMG_OK : DGMG_EHIP;
}

template <class A>
BatchList<A> blist(dgmg_batch* b, const dgmg_batch::Launch& ln) {
  BatchList<A> bl;
  bl.descs = (const A*)(b->ws + b->plan_off + ln.desc_off);
  bl.starts = (const int*)(b->ws + b->plan_off + ln.starts_off);
  bl.ng = ln.ng;
  return bl;
}

template <class T, int DIM>
int run_launch_t(dgmg_batch* b, const dgmg_batch::Launch& ln, hipStream_t s) {
  switch (ln.kind) {
    case BK_APPLY: return Kern<T, DIM>::apply_batch(ln.t[0], ln.t[1], blist<ApplyArgs<T>>(b, ln), ln.ntot, s);
    case BK_FDM: return Kern<T, DIM>::fdm_batch(ln.t[0], ln.t[1], ln.t[2], blist<FdmArgs<T>>(b, ln), ln.ntot, 0, s);
    case BK_COMB: return Kern<T, DIM>::combine_batch(ln.t[0], ln.t[1], blist<CombArgs<T>>(b, ln), ln.ntot, s);
    case BK_XFER:
      return Kern<T, DIM>::transfer_batch(ln.t[0], ln.t[1], ln.t[2] != 0, blist<XferArgs<T>>(b, ln), ln.ntot, s);
    default: return -4;
  }
}

// skip_done: leave out the per-grid operations of grids that have converged
// (eager runs; a recorded graph keeps them, and their kernels return at once)
int run_plan(dgmg_batch* b, int which, hipStream_t s, bool skip_done) {
  const auto& plan = b->plan[which];
  std::vector<int> act;
  for (size_t i0 = 0; i0 < plan.size();) {
    // the launches of one plan position touch disjoint grids: with side
    // streams, the per-grid steps (round robin over the side streams) overlap
    // the position's work-list launches on s, joined before the next position
    size_t i1 = i0 + 1;
    while (i1 < plan.size() && plan[i1].key == plan[i0].key) ++i1;
    int used = 0;  // side streams forked at this position
    for (size_t li = i0; li < i1; ++li) {
      const auto& ln = plan[li];
      if (ln.kind != BK_FN) continue;
      act.clear();
      for (size_t k = 0; k < ln.fns.size(); ++k)
        if (!skip_done || b->flags_host[ln.fn_grid[k]]) act.push_back((int)k);
      const int ns = b->concurrent ? std::min<int>(b->nside, (int)act.size()) : 0;
      if (ns == 0) {
        for (int k : act) {
          int rc = ln.fns[k]();
          if (rc) return rc;
        }
        continue;
      }
      if (used == 0) {
        if (hipEventRecord(b->ev_fork, s) != hipSuccess) return DGMG_EHIP;
        for (int i = 0; i < b->nside; ++i)
          if (hipStreamWaitEvent(b->side[i], b->ev_fork, 0) != hipSuccess) return DGMG_EHIP;
        used = b->nside;
      }
      for (size_t j = 0; j < act.size(); ++j) {
        dgmg_handle* h = b->h[ln.fn_grid[act[j]]];
        const hipStream_t keep = h->stream;
        h->stream = b->side[j % ns];
        const int rc = ln.fns[act[j]]();
        h->stream = keep;
        if (rc) return rc;
      }
    }
    for (size_t li = i0; li < i1; ++li) {
      const auto& ln = plan[li];
      if (ln.kind == BK_FN) continue;
      int rc;
      if (ln.f32) rc = ln.dim == 3 ? run_launch_t<float, 3>(b, ln, s) : run_launch_t<float, 2>(b, ln, s);
      else rc = ln.dim == 3 ? run_launch_t<double, 3>(b, ln, s) : run_launch_t<double, 2>(b, ln, s);
      if (rc) return DGMG_EUNSUPPORTED;
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return DGMG_EHIP;
    }
    for (int i = 0; i < used; ++i) {
      if (hipEventRecord(b->ev_join[i], b->side[i]) != hipSuccess) return DGMG_EHIP;
      if (hipStreamWaitEvent(s, b->ev_join[i], 0) != hipSuccess) return DGMG_EHIP;
    }
    i0 = i1;
  }
  return DGMG_OK;
}

}  // namespace

extern "C" {

// ------------------------------------------------------------------- batches
int dgmg_batch_setup(int count, const dgmg_grid* grids, const dgmg_opts* opts, dgmg_batch** out) {
  if (!out || count < 1 || !grids || !opts) return fail(nullptr, DGMG_EINVAL, "bad batch arguments");
  *out = nullptr;
  dgmg_batch* b = new dgmg_batch();
  Carver cv{nullptr};
  cv.take(count * sizeof(int));
  cv.take(count * sizeof(double));
  b->dof_off.push_back(0);
  for (int i = 0; i < count; ++i) {
    dgmg_handle* h = nullptr;
    int rc = dgmg_setup(&grids[i], &opts[i], &h);
    if (rc) {
      for (auto* x : b->h) dgmg_destroy(x);
      delete b;
      g_setup_error = "grid " + std::to_string(i) + ": " + g_setup_error;
      return rc;
    }
    b->h.push_back(h);
    if (h->sp.disc != DGMG_DISC_DG) {
      for (auto* x : b->h) dgmg_destroy(x);
      delete b;
      return fail(nullptr, DGMG_EUNSUPPORTED, "grid " + std::to_string(i) + ": batches take DG grids only");
    }
    cv.off = (cv.off + 255) & ~size_t(255);  // member workspaces: 256-aligned, disjoint
    b->sub_off.push_back(cv.off);
    cv.off += h->ws_need;
    b->dof_off.push_back(b->dof_off.back() + h->lv.back().n_dof);
  }
  // the batched execution plan's descriptors (sized by a dry run)
  batch_plan(b, false);
  if (b->planned) {
    cv.off = (cv.off + 255) & ~size_t(255);
    b->plan_off = cv.off;
    cv.off += b->plan_bytes;
  }
  b->ws_need = cv.off + 256;
  *out = b;
  return DGMG_OK;
}

int dgmg_batch_plan_info(const dgmg_batch* b, int* planned, int* kernels, int* grid_ops) {
  if (!b) return DGMG_EINVAL;
  int k = 0, g = 0;
  for (const auto& ph : b->plan)
    for (const auto& ln : ph) {
      if (ln.kind == BK_FN) g += (int)ln.fns.size();
      else ++k;
    }
  if (planned) *planned = b->planned ? 1 : 0;
  if (kernels) *kernels = k;
  if (grid_ops) *grid_ops = g;
  return DGMG_OK;
}

int dgmg_batch_workspace_bytes(const dgmg_batch* b, size_t* bytes) {
  if (!b || !bytes) return DGMG_EINVAL;
  *bytes = b->ws_need;
  return DGMG_OK;
}

int dgmg_batch_offsets(const dgmg_batch* b, int64_t* offsets) {
  if (!b || !offsets) return DGMG_EINVAL;
  for (size_t i = 0; i < b->dof_off.size(); ++i) offsets[i] = b->dof_off[i];
  return DGMG_OK;
}

int dgmg_batch_handle(dgmg_batch* b, int i, dgmg_handle** h) {
  if (!b || !h || i < 0 || i >= (int)b->h.size()) return DGMG_EINVAL;
  *h = b->h[i];
  return DGMG_OK;
}

int dgmg_batch_bind_workspace(dgmg_batch* b, void* dev, size_t bytes, void* stream) {
  if (!b || !dev) return DGMG_EINVAL;
  if (bytes < b->ws_need) {
    b->err = "workspace too small";
    return DGMG_ENOMEM;
  }
  if (((uintptr_t)dev) & 255) {
    b->err = "workspace must be 256-byte aligned";
    return DGMG_EINVAL;
  }
  for (auto& g : b->gexec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  b->stream = (hipStream_t)stream;
  b->ws = (char*)dev;
  const int n = (int)b->h.size();
  Carver cv{b->ws};
  b->flags_dev = (int*)cv.take(n * sizeof(int));
  b->rr_dev = (double*)cv.take(n * sizeof(double));
  if (!b->flags_host) {
    if (hipHostMalloc((void**)&b->flags_host, n * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&b->rr_host, n * sizeof(double), hipHostMallocDefault) != hipSuccess) {
      b->err = "pinned alloc failed";
      return DGMG_EHIP;
    }
  }
  // every member range must lie after the header, be aligned and end before the next one
  size_t prev_end = cv.off;
  for (int i = 0; i < n; ++i) {
    const size_t lo = b->sub_off[i], hi = lo + b->h[i]->ws_need;
    if (lo < prev_end || (lo & 255) || hi > b->ws_need) {
      b->err = "internal: batch workspace layout is inconsistent";
      return DGMG_EINVAL;
    }
    prev_end = hi;
  }
  for (int i = 0; i < n; ++i) {
    int rc = bind_batch_member(b->h[i], b->ws + b->sub_off[i], b->stream, b->flags_dev + i, b->rr_dev + i);
    if (rc) {
      b->err = "grid " + std::to_string(i) + ": " + b->h[i]->err;
      return rc;
    }
  }
  if (b->planned && b->nside == 0) {  // side streams (default priority) and their events, once
    bool ok = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; ok && i < dgmg_batch::NSIDE; ++i)
      ok = hipStreamCreateWithFlags(&b->side[i], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&b->ev_join[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      b->err = "side stream creation failed";
      return DGMG_EHIP;
    }
    b->nside = dgmg_batch::NSIDE;
  }
  if (b->planned) {
    if (b->plan_off < prev_end || b->plan_off + b->plan_bytes > b->ws_need) {
      b->err = "internal: batch plan region is inconsistent";
      return DGMG_EINVAL;
    }
    int rc = batch_plan(b, true);
    if (rc) {
      b->err = "batch plan upload failed";
      return rc;
    }
  }
  b->bound = true;
  return DGMG_OK;
}

static int batch_fail(dgmg_batch* b, int code, const std::string& msg) {
  b->err = msg;
  return code;
}

static int batch_flags_upload(dgmg_batch* b) {
  hipError_t e = hipMemcpyAsync(b->flags_dev, b->flags_host, b->h.size() * sizeof(int), hipMemcpyHostToDevice,
                                b->stream);
  return e == hipSuccess ? DGMG_OK : batch_fail(b, DGMG_EHIP, std::string("flag upload: ") + hipGetErrorString(e));
}

static int batch_rr_download(dgmg_batch* b) {
  hipError_t e = hipMemcpyAsync(b->rr_host, b->rr_dev, b->h.size() * sizeof(double), hipMemcpyDeviceToHost,
                                b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  return e == hipSuccess ? DGMG_OK : batch_fail(b, DGMG_EHIP, std::string("norm readback: ") + hipGetErrorString(e));
}

int dgmg_batch_autotune(dgmg_batch* b) {
  if (!b || !b->bound) return DGMG_EINVAL;
  for (size_t i = 0; i < b->h.size(); ++i) b->flags_host[i] = 1;
  int rc = batch_flags_upload(b);
  if (rc) return rc;
  // grids whose sweeps have the same tile and patch counts share one measurement
  std::vector<std::pair<std::vector<int64_t>, int>> seen;
  for (dgmg_handle* h : b->h) {
    for (int l = 1; l < (int)h->lv.size(); ++l) {
      const int nk = ec_smoother(h) ? 1 : h->lv[l].dim;
      for (int q = 0; q < nk; ++q) {
        const int nd = ec_smoother(h) ? -1 : q;
        int np[3], NA, NL;
        sweep_shape(h->lv[l], nd, np, NA, NL);
        std::vector<int64_t> key{(int64_t)mg_size(h), h->lv[l].dim, NA, NL, np[0], np[1], np[2]};
        int found = -1;
        for (auto& s : seen)
          if (s.first == key) found = s.second;
        if (found >= 0) {
          h->waves[l][nd < 0 ? 3 : nd] = found;
          continue;
        }
        seen.emplace_back(key, -1);
        // tune this handle's level fully, then record the choice of this sweep
        int keep[NKIND];
        for (int k = 0; k < NKIND; ++k) keep[k] = h->waves[l][k];
        hipEvent_t e0, e1;
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        float best = 1e30f;
        int bw = 0;
        for (int w : {1, 2, 4, 8}) {
          const bool f32 = mixed(h);
          auto launch = [&]() {
            return f32 ? k_fdm<float>(h, l, nd, (const float*)h->buf[l].r, w)
                       : k_fdm<double>(h, l, nd, (const double*)h->buf[l].r, w);
          };
          if (f32) k_fill_v<float>(h, (float*)h->buf[l].r, h->lv[l].n_dof);
          else k_fill_v<double>(h, (double*)h->buf[l].r, h->lv[l].n_dof);
          if ((rc = launch())) break;
          (void)hipEventRecord(e0, h->stream);
          for (int rep = 0; rep < 3 && !rc; ++rep) rc = launch();
          (void)hipEventRecord(e1, h->stream);
          if (rc || hipEventSynchronize(e1) != hipSuccess) {
            rc = rc ? rc : DGMG_EHIP;
            break;
          }
          float ms = 0;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (ms < best) {
            best = ms;
            bw = w;
          }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) return batch_fail(b, rc, "autotune: " + h->err);
        for (int k = 0; k < NKIND; ++k) h->waves[l][k] = keep[k];
        h->waves[l][nd < 0 ? 3 : nd] = bw;
        h->tune_ms[l][nd < 0 ? 3 : nd] = best / 3.0f;
        seen.back().second = bw;
      }
    }
    drop_graphs(h);
  }
  for (auto& g : b->gexec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  return DGMG_OK;
}

int dgmg_batch_use_graphs(dgmg_batch* b, int enable) {
  if (!b) return DGMG_EINVAL;
  for (auto& g : b->gexec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  b->use_graphs = enable != 0;
  return DGMG_OK;
}

// One MGCG phase for every grid: a graph whose per-grid chains are independent
// child graphs (captured once, replayed each iteration; converged grids are
// masked by their device flag), or eager launches.
// The planned phase (launches over work lists), recorded into one graph per
// phase and x, or run directly.
static int batch_phase_planned(dgmg_batch* b, int which, double* x) {
  b->x_cur = x;
  if (!b->use_graphs) {
    int rc = run_plan(b, which, b->stream, true);
    return rc ? batch_fail(b, rc, "batched launch failed") : DGMG_OK;
  }
  if (which == 0 && b->gexec[0] && b->graph_x != x) {
    (void)hipGraphExecDestroy(b->gexec[0]);
    b->gexec[0] = nullptr;
  }
  if (!b->gexec[which]) {
    if (!b->cap_stream) {
      hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return batch_fail(b, DGMG_EHIP, std::string("capture stream: ") + hipGetErrorString(e));
    }
    hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return batch_fail(b, DGMG_EHIP, std::string("begin capture: ") + hipGetErrorString(e));
    for (auto* h : b->h) h->stream = b->cap_stream;
    int rc = run_plan(b, which, b->cap_stream, false);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap_stream, &g);
    for (auto* h : b->h) h->stream = b->stream;
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return batch_fail(b, rc, "batched launch failed");
    }
    if (e != hipSuccess) return batch_fail(b, DGMG_EHIP, std::string("end capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&b->gexec[which], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return batch_fail(b, DGMG_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    if (which == 0) b->graph_x = x;
  }
  hipError_t e = hipGraphLaunch(b->gexec[which], b->stream);
  return e == hipSuccess ? DGMG_OK : batch_fail(b, DGMG_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
}

static int batch_phase(dgmg_batch* b, int which, double* x) {
  const int n = (int)b->h.size();
  if (b->planned) return batch_phase_planned(b, which, x);
  if (!b->use_graphs) {
    for (int i = 0; i < n; ++i) {
      int rc = which == 0 ? pcg_phase_a(b->h[i], x + b->dof_off[i]) : pcg_phase_b(b->h[i]);
      if (rc) return batch_fail(b, rc, "grid " + std::to_string(i) + ": " + b->h[i]->err);
    }
    return DGMG_OK;
  }
  if (which == 0 && b->gexec[0] && b->graph_x != x) {
    (void)hipGraphExecDestroy(b->gexec[0]);
    b->gexec[0] = nullptr;
  }
  if (!b->gexec[which]) {
    hipGraph_t parent = nullptr;
    if (hipGraphCreate(&parent, 0) != hipSuccess) return batch_fail(b, DGMG_EHIP, "graph create");
    for (int i = 0; i < n; ++i) {
      dgmg_handle* h = b->h[i];
      hipGraph_t g = nullptr;
      double* xi = x + b->dof_off[i];
      int rc = capture(h, &g, [&]() { return which == 0 ? pcg_phase_a(h, xi) : pcg_phase_b(h); });
      if (rc) {
        (void)hipGraphDestroy(parent);
        return batch_fail(b, rc, "grid " + std::to_string(i) + ": " + h->err);
      }
      hipGraphNode_t node;
      hipError_t e = hipGraphAddChildGraphNode(&node, parent, nullptr, 0, g);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(parent);
        return batch_fail(b, DGMG_EHIP, std::string("child graph: ") + hipGetErrorString(e));
      }
    }
    hipError_t e = hipGraphInstantiate(&b->gexec[which], parent, nullptr, nullptr, 0);
    (void)hipGraphDestroy(parent);
    if (e != hipSuccess) return batch_fail(b, DGMG_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    if (which == 0) b->graph_x = x;
  }
  hipError_t e = hipGraphLaunch(b->gexec[which], b->stream);
  return e == hipSuccess ? DGMG_OK : batch_fail(b, DGMG_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
}

int dgmg_batch_solve(dgmg_batch* b, const double* rhs, double* x, double tol, dgmg_stats* st) {
  if (!b || !rhs || !x || !(tol >= 0)) return DGMG_EINVAL;
  if (!b->bound) return batch_fail(b, DGMG_ENOMEM, "workspace not bound");
  const int n = (int)b->h.size();
  std::vector<double> r0(n), rmax(n), rn(n);
  std::vector<int> its(n, 0), conv(n, 0);
  if (st) std::memset(st, 0, sizeof(dgmg_stats) * n);
  for (int i = 0; i < n; ++i) b->flags_host[i] = 1;
  int rc = batch_flags_upload(b);
  if (rc) return rc;
  for (int i = 0; i < n; ++i)
    if ((rc = check_rhs_consistent(b->h[i], rhs + b->dof_off[i])))
      return batch_fail(b, rc, "grid " + std::to_string(i) + ": " + b->h[i]->err);
  for (int i = 0; i < n; ++i)
    if ((rc = pcg_init_a(b->h[i], rhs + b->dof_off[i], x + b->dof_off[i])))
      return batch_fail(b, rc, "grid " + std::to_string(i) + ": " + b->h[i]->err);
  if ((rc = batch_rr_download(b))) return rc;
  int maxit = 0;
  for (int i = 0; i < n; ++i) {
    r0[i] = std::sqrt(b->rr_host[i]);
    if (!std::isfinite(r0[i])) return batch_fail(b, DGMG_ENONFINITE, "grid " + std::to_string(i) + ": initial residual not finite");
    rmax[i] = tol * r0[i];
    rn[i] = r0[i];
    conv[i] = r0[i] == 0.0;
    b->flags_host[i] = conv[i] ? 0 : 1;
    maxit = std::max(maxit, b->h[i]->opts.max_iter);
    if (st) {
      st[i].r0 = r0[i];
      st[i].r_final = r0[i];
      st[i].history[0] = r0[i];
      st[i].converged = conv[i];
    }
  }
  if ((rc = batch_flags_upload(b))) return rc;
  for (int i = 0; i < n; ++i)
    if ((rc = pcg_init_b(b->h[i]))) return batch_fail(b, rc, "grid " + std::to_string(i) + ": " + b->h[i]->err);
  for (int it = 1; it <= maxit; ++it) {
    bool any = false;
    for (int i = 0; i < n; ++i) any = any || b->flags_host[i];
    if (!any) break;
    if ((rc = batch_phase(b, 0, x))) return rc;
    if ((rc = batch_rr_download(b))) return rc;
    any = false;
    for (int i = 0; i < n; ++i) {
      if (!b->flags_host[i]) continue;
      its[i] = it;
      rn[i] = std::sqrt(b->rr_host[i]);
      if (st) {
        st[i].iterations = it;
        st[i].r_final = rn[i];
        if (it < 256) st[i].history[it] = rn[i];
      }
      if (!std::isfinite(rn[i])) return batch_fail(b, DGMG_ENONFINITE, "grid " + std::to_string(i) + ": residual not finite");
      bool done = false;
      if (rn[i] <= rmax[i]) {
        // exit confirmation on the true residual, as for a single solve (the
        // grid's device flag is still set, so its kernels run)
        double rt;
        if ((rc = true_residual(b->h[i], rhs + b->dof_off[i], x + b->dof_off[i], &rt)))
          return batch_fail(b, rc, "grid " + std::to_string(i) + ": " + b->h[i]->err);
        if (st) st[i].r_true = rt;
        done = rt <= rmax[i];
        if (!done && st) st[i].replacements++;
      }
      if (done) {
        conv[i] = 1;
        b->flags_host[i] = 0;
      } else if (it >= b->h[i]->opts.max_iter) {
        b->flags_host[i] = 0;
      } else {
        any = true;
      }
    }
    if (!any) break;
    if ((rc = batch_flags_upload(b))) return rc;
    if ((rc = batch_phase(b, 1, x))) return rc;
  }
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return batch_fail(b, DGMG_EHIP, hipGetErrorString(e));
  bool all = true;
  for (int i = 0; i < n; ++i) {
    all = all && conv[i];
    if (st) {
      st[i].converged = conv[i];
      if (its[i] > 0) st[i].rho = std::pow(rn[i] / r0[i], 1.0 / its[i]);
    }
  }
  return all ? DGMG_OK : DGMG_NOT_CONVERGED;
}

const char* dgmg_batch_last_error(const dgmg_batch* b) { return b ? b->err.c_str() : g_setup_error.c_str(); }

void dgmg_batch_destroy(dgmg_batch* b) {
  if (!b) return;
  for (auto& g : b->gexec)
    if (g) (void)hipGraphExecDestroy(g);
  for (auto* h : b->h) dgmg_destroy(h);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (int i = 0; i < dgmg_batch::NSIDE; ++i) {
    if (b->side[i]) (void)hipStreamDestroy(b->side[i]);
    if (b->ev_join[i]) (void)hipEventDestroy(b->ev_join[i]);
  }
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->flags_host) (void)hipHostFree(b->flags_host);
  if (b->rr_host) (void)hipHostFree(b->rr_host);
  delete b;
}

}  // extern "C"

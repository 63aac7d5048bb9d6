// C ABI of the gfx950 DG p-multigrid solver: handle, workspace, coarse solve,
// PCG vector kernels and the orchestration of Alg. 1 (V-cycle) and Alg. 2 (MGCG).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dgmg.h"
#include "kernels.hpp"
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

constexpr int RED_BLOCKS = 1024;  // fixed partial count of the vector reductions
constexpr int VEC_THREADS = 256;

// ---------------------------------------------------------------- vector kernels (FP64 PCG)
__global__ void __launch_bounds__(VEC_THREADS) k_dot(const double* __restrict__ a,
                                                     const double* __restrict__ b, int64_t n,
                                                     double* __restrict__ part) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += a[i] * b[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Sum of partials in a fixed order into out[0] (one block).
__global__ void __launch_bounds__(VEC_THREADS) k_finalize(const double* __restrict__ part, int np,
                                                          double* __restrict__ out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = s;
}

// z.(r - r_old) and z.r partials.
__global__ void __launch_bounds__(VEC_THREADS) k_dot_zr(const double* __restrict__ z,
                                                        const double* __restrict__ r,
                                                        const double* __restrict__ ro, int64_t n,
                                                        double* __restrict__ part1,
                                                        double* __restrict__ part2) {
  __shared__ double red[16];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double zi = z[i], ri = r[i];
    s1 += zi * (ri - ro[i]);
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

// alpha = delta / (p.q); x += alpha p; r -= alpha q; partial r.r
__global__ void __launch_bounds__(VEC_THREADS) k_update_xr(double* __restrict__ x, double* __restrict__ r,
                                                           const double* __restrict__ p,
                                                           const double* __restrict__ q,
                                                           const double* __restrict__ delta,
                                                           const double* __restrict__ pq, int64_t n,
                                                           double* __restrict__ part) {
  __shared__ double red[16];
  const double alpha = delta[0] / pq[0];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    s += ri * ri;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// beta = num / delta_old; p = z + beta p; r_old = r
__global__ void __launch_bounds__(VEC_THREADS) k_update_p(double* __restrict__ p, const double* __restrict__ z,
                                                          const double* __restrict__ r,
                                                          double* __restrict__ ro,
                                                          const double* __restrict__ num,
                                                          const double* __restrict__ delta_old,
                                                          int64_t n) {
  const double beta = num[0] / delta_old[0];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    p[i] = z[i] + beta * p[i];
    ro[i] = r[i];
  }
}

template <class A, class B>
__global__ void __launch_bounds__(VEC_THREADS) k_convert(const A* __restrict__ a, B* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (B)a[i];
}

template <class T>
__global__ void __launch_bounds__(VEC_THREADS) k_fill(T* __restrict__ a, T v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

__global__ void __launch_bounds__(VEC_THREADS) k_copy(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// a -= s[0] * scale
__global__ void __launch_bounds__(VEC_THREADS) k_sub_scalar(double* __restrict__ a, const double* __restrict__ s,
                                                            double scale, int64_t n) {
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
  int N[3];
  const double* S[3];    // G_d x G_d row-major
  const double* lam[3];  // G_d
};

template <bool FWD, bool SCALE>
__global__ void __launch_bounds__(VEC_THREADS) k_coarse_pass(CoarseDev C, int d, const double* __restrict__ in,
                                                             double* __restrict__ out, int64_t n) {
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
  for (int K = 0; K < G; ++K) {
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

inline unsigned vec_blocks(int64_t n) {
  int64_t b = (n + VEC_THREADS - 1) / VEC_THREADS;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

}  // namespace

// =================================================================== handle
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
  std::vector<Bufs> buf;  // per level, MG precision
  void* patch = nullptr;  // patch buffer (MG precision), also used by dgmg_smooth in either precision
  size_t patch_elems = 0;
  double *c_a = nullptr, *c_b = nullptr, *c_f = nullptr;  // coarse FDM scratch (FP64)
  CoarseDev cdev{};
  // PCG (top level, FP64)
  double *pr = nullptr, *pro = nullptr, *pp = nullptr, *pq = nullptr, *pz = nullptr;
  double* part = nullptr;   // 2 * RED_BLOCKS
  double* scal = nullptr;   // scalar slots
  double* host_scal = nullptr;  // pinned
  // timing
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  std::vector<double> ev_flops, ev_bytes;
  double t_ms = 0, t_flops = 0, t_bytes = 0;
  int64_t t_launch = 0;
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

template <class T>
void carve_level(Carver& cv, const LevelHost& h, LevelDev<T>& d, std::vector<std::pair<void*, std::vector<char>>>* up) {
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
  d.dim = h.dim;
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
    dd.n_ec = s.n_ec;
    dd.n_fc = s.n_fc;
    dd.nf = s.nf;
    dd.ecoef = put(s.ecoef);
    dd.nbr = put_int(s.nbr);
    if (!s.S_ec.empty()) {
      auto transp = [](const std::vector<double>& S, int n) {
        std::vector<double> t(S.size());
        const size_t nb = S.size() / ((size_t)n * n);
        for (size_t b = 0; b < nb; ++b)
          for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) t[b * n * n + (size_t)j * n + i] = S[b * n * n + (size_t)i * n + j];
        return t;
      };
      dd.ST_ec = put(transp(s.S_ec, s.n_ec));
      dd.ST_fc = put(transp(s.S_fc, s.n_fc));
      dd.S_ec = put(s.S_ec);
      dd.lam_ec = put(s.lam_ec);
      dd.w_ec = put(s.w_ec);
      dd.S_fc = put(s.S_fc);
      dd.lam_fc = put(s.lam_fc);
      dd.w_fc = put(s.w_fc);
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

int layout(dgmg_handle* h, char* base, std::vector<std::pair<void*, std::vector<char>>>* up) {
  Carver cv{base};
  const int nl = (int)h->lv.size();
  h->Ld.assign(nl, LevelDev<double>());
  h->Lf.assign(nl, LevelDev<float>());
  for (int l = 0; l < nl; ++l) {
    carve_level<double>(cv, h->lv[l], h->Ld[l], up);
    carve_level<float>(cv, h->lv[l], h->Lf[l], up);
  }
  // coarse global eigenpairs
  const LevelHost& l0 = h->lv[0];
  h->cdev.dim = l0.dim;
  for (int d = 0; d < 3; ++d) {
    h->cdev.N[d] = d < l0.dim ? l0.dir[d].N : 1;
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
  const size_t apply_blocks = h->lv.back().n_elem + 8;
  h->part = (double*)cv.take(std::max<size_t>(2 * RED_BLOCKS, apply_blocks) * 8 + 2 * RED_BLOCKS * 8);
  h->scal = (double*)cv.take(64 * 8);
  h->ws_need = cv.off + 256;
  return DGMG_OK;
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
  int rc = L.dim == 3 ? Kern<T, 3>::apply(L, mode, x, f, y, part, nb, h->stream)
                      : Kern<T, 2>::apply(L, mode, x, f, y, part, nb, h->stream);
  if (rc) return fail(h, DGMG_EUNSUPPORTED, "no operator kernel for this order");
  return check_hip(h, "apply");
}

template <class T>
int k_sweep(dgmg_handle* h, int l, int nd, T* u, const T* f, T* r) {
  const LevelDev<T>& L = LD<T>(h, l);
  const LevelHost& lv = h->lv[l];
  int rc = k_apply<T>(h, l, 1, u, f, r, nullptr, nullptr);
  if (rc) return rc;
  int np[3] = {1, 1, 1};
  for (int d = 0; d < lv.dim; ++d) np[d] = (d == nd) ? lv.dir[d].nf : lv.dir[d].N;
  const int NL = lv.NP + 2 * lv.NO;
  const int NA = nd < 0 ? NL : 2 * lv.P;
  T* pb = (T*)h->patch;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timed = h->timing && l == (int)h->lv.size() - 1;  // top-level launches only
  if (timed) {
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventRecord(e0, h->stream);
  }
  rc = L.dim == 3 ? Kern<T, 3>::fdm(L, nd, NA, NL, r, pb, np[0], np[1], np[2], h->stream)
                  : Kern<T, 2>::fdm(L, nd, NA, NL, r, pb, np[0], np[1], np[2], h->stream);
  if (rc) return fail(h, DGMG_EUNSUPPORTED, "no patch-solve kernel for this tile");
  if (timed) {
    (void)hipEventRecord(e1, h->stream);
    h->ev.emplace_back(e0, e1);
    // algorithmic cost of one launch: 2 flops per multiply-add of the 2D
    // forward and backward 1D contractions, plus scale and weight; bytes:
    // residual read + weighted correction written, per patch tile
    double npatch = (double)np[0] * np[1] * np[2];
    double ts = NA, fl = 0.0;
    for (int d = 1; d < lv.dim; ++d) ts *= NL;
    fl = 2.0 * 2.0 * ts * (NA + (lv.dim - 1) * NL) + 2.0 * ts;
    h->ev_flops.push_back(npatch * fl);
    h->ev_bytes.push_back(npatch * ts * 2.0 * sizeof(T));
  }
  rc = check_hip(h, "patch solve");
  if (rc) return rc;
  rc = L.dim == 3 ? Kern<T, 3>::combine(L, nd, NA, NL, pb, u, np[0], np[1], np[2], h->stream)
                  : Kern<T, 2>::combine(L, nd, NA, NL, pb, u, np[0], np[1], np[2], h->stream);
  if (rc) return fail(h, DGMG_EUNSUPPORTED, "no combine kernel for this order");
  return check_hip(h, "combine");
}

template <class T>
int k_smooth(dgmg_handle* h, int l, T* u, const T* f, int steps, T* r) {
  for (int s = 0; s < steps; ++s) {
    if (h->opts.smoother == DGMG_SMOOTHER_EA) {
      int rc = k_sweep<T>(h, l, -1, u, f, r);
      if (rc) return rc;
    } else {
      for (int d = 0; d < h->lv[l].dim; ++d) {
        int rc = k_sweep<T>(h, l, d, u, f, r);
        if (rc) return rc;
      }
    }
  }
  return DGMG_OK;
}

template <class T>
int k_transfer(dgmg_handle* h, int l, bool restr, const T* in, T* out) {
  const LevelDev<T>& L = LD<T>(h, l);
  int rc = L.dim == 3 ? Kern<T, 3>::transfer(L, restr, in, out, h->stream)
                      : Kern<T, 2>::transfer(L, restr, in, out, h->stream);
  if (rc) return fail(h, DGMG_EUNSUPPORTED, "no transfer kernel for this order pair");
  return check_hip(h, "transfer");
}

template <class T>
void k_fill_v(dgmg_handle* h, T* a, int64_t n) {
  hipLaunchKernelGGL(k_fill<T>, dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, a, T(0), n);
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
    hipLaunchKernelGGL(k_copy, dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, f0, h->c_f, n);
    hipLaunchKernelGGL(k_fill<double>, dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, h->c_a, 1.0, n);
    hipLaunchKernelGGL(k_dot, dim3(RED_BLOCKS), dim3(VEC_THREADS), 0, h->stream, h->c_f, h->c_a, n, h->part);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(VEC_THREADS), 0, h->stream, h->part, RED_BLOCKS, h->scal + 41);
    hipLaunchKernelGGL(k_sub_scalar, dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, h->c_f, h->scal + 41, 1.0 / (double)n, n);
    src = h->c_f;
  }
  double* a = h->c_a;
  double* b = h->c_b;
  // forward passes x, y, (z with scale)
  const double* in = src;
  double* bufs[2] = {a, b};
  int k = 0;
  for (int d = 0; d < dim; ++d) {
    double* out = bufs[k];
    if (d == dim - 1)
      hipLaunchKernelGGL((k_coarse_pass<true, true>), dim3(nb), dim3(VEC_THREADS), 0, h->stream, h->cdev, d, in, out, n);
    else
      hipLaunchKernelGGL((k_coarse_pass<true, false>), dim3(nb), dim3(VEC_THREADS), 0, h->stream, h->cdev, d, in, out, n);
    in = out;
    k ^= 1;
  }
  for (int d = dim - 1; d >= 0; --d) {
    double* out = d == 0 ? u0 : bufs[k];
    hipLaunchKernelGGL((k_coarse_pass<false, false>), dim3(nb), dim3(VEC_THREADS), 0, h->stream, h->cdev, d, in, out, n);
    in = out;
    k ^= 1;
  }
  if (periodic_all) {  // mean-free (minimum-norm) representative
    hipLaunchKernelGGL(k_fill<double>, dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, h->c_a, 1.0, n);
    hipLaunchKernelGGL(k_dot, dim3(RED_BLOCKS), dim3(VEC_THREADS), 0, h->stream, u0, h->c_a, n, h->part);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(VEC_THREADS), 0, h->stream, h->part, RED_BLOCKS, h->scal + 41);
    hipLaunchKernelGGL(k_sub_scalar, dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, u0, h->scal + 41, 1.0 / (double)n, n);
  }
  return check_hip(h, "coarse solve");
}

template <class T>
int k_coarse(dgmg_handle* h, const T* f0, T* u0);
template <>
int k_coarse<double>(dgmg_handle* h, const double* f0, double* u0) { return coarse_fdm(h, f0, u0); }
template <>
int k_coarse<float>(dgmg_handle* h, const float* f0, float* u0) {
  const int64_t n = h->lv[0].n_dof;
  // FP64 copies: input in the level-0 residual buffer (sized for doubles),
  // result in the patch buffer (c_a, c_b and c_f are used by coarse_fdm)
  double* tmp_in = (double*)h->buf[0].r;
  double* res = (double*)h->patch;
  hipLaunchKernelGGL((k_convert<float, double>), dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, f0, tmp_in, n);
  int rc = coarse_fdm(h, tmp_in, res);
  if (rc) return rc;
  hipLaunchKernelGGL((k_convert<double, float>), dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, res, u0, n);
  return check_hip(h, "coarse convert");
}

// z = MultigridCycle(0, r) on MG-precision vectors (Alg. 1).
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
    int base = which == 0 ? h->opts.ns_pre : h->opts.ns_post;
    return var ? base << (L - l) : base;
  };
  k_fill_v<T>(h, u[L], h->lv[L].n_dof);
  for (int l = L; l >= 1; --l) {
    if (l < L) k_fill_v<T>(h, u[l], h->lv[l].n_dof);
    T* rl = (T*)h->buf[l].r;
    int rc = k_smooth<T>(h, l, u[l], f[l], ns(l, 0), rl);
    if (rc) return rc;
    rc = k_apply<T>(h, l, 1, u[l], f[l], rl, nullptr, nullptr);
    if (rc) return rc;
    rc = k_transfer<T>(h, l, true, rl, f[l - 1]);
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
int precond(dgmg_handle* h, const double* r, double* z) {
  const int L = (int)h->lv.size() - 1;
  const int64_t n = h->lv[L].n_dof;
  if (!mixed(h)) return k_vcycle<double>(h, r, z);
  float* rf = (float*)h->buf[L].f;
  float* zf = (float*)h->buf[L].u;
  hipLaunchKernelGGL((k_convert<double, float>), dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, r, rf, n);
  int rc = k_vcycle<float>(h, rf, zf);
  if (rc) return rc;
  hipLaunchKernelGGL((k_convert<float, double>), dim3(vec_blocks(n)), dim3(VEC_THREADS), 0, h->stream, zf, z, n);
  return check_hip(h, "precond convert");
}

int read_scalar(dgmg_handle* h, const double* dev, double* out) {
  hipError_t e = hipMemcpyAsync(h->host_scal, dev, sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(h, DGMG_EHIP, std::string("scalar readback: ") + hipGetErrorString(e));
  *out = *h->host_scal;
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
  if (!g || !o || !out) return fail(nullptr, DGMG_EINVAL, "null argument");
  *out = nullptr;
  if (g->dim != 2 && g->dim != 3) return fail(nullptr, DGMG_EINVAL, "dim must be 2 or 3");
  const int okP[] = {1, 2, 3, 4, 6, 8, 12, 16};
  if (std::find(std::begin(okP), std::end(okP), o->P) == std::end(okP))
    return fail(nullptr, DGMG_EUNSUPPORTED, "P must be one of 1, 2, 3, 4, 6, 8, 12, 16");
  if (!(o->mu_star > 0) || !std::isfinite(o->mu_star)) return fail(nullptr, DGMG_EINVAL, "mu_star must be > 0");
  if (o->flux != DGMG_FLUX_IP && o->flux != DGMG_FLUX_LDG) return fail(nullptr, DGMG_EINVAL, "bad flux");
  if (o->smoother != DGMG_SMOOTHER_EA && o->smoother != DGMG_SMOOTHER_FA) return fail(nullptr, DGMG_EINVAL, "bad smoother");
  if (o->weighting < 0 || o->weighting > 3) return fail(nullptr, DGMG_EINVAL, "bad weighting");
  if (o->vcycle != DGMG_VCYCLE_CLASSICAL && o->vcycle != DGMG_VCYCLE_VARIABLE) return fail(nullptr, DGMG_EINVAL, "bad vcycle");
  if (o->precision != DGMG_PREC_FP64 && o->precision != DGMG_PREC_MIXED) return fail(nullptr, DGMG_EINVAL, "bad precision");
  if (o->ns_pre < 0 || o->ns_post < 0 || o->max_iter < 0) return fail(nullptr, DGMG_EINVAL, "negative count");
  if (o->overlap < -2) return fail(nullptr, DGMG_EINVAL, "bad overlap");
  SetupParams sp;
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
  if (ne * (int64_t)std::pow(o->P + 1, g->dim) > (int64_t)INT32_MAX * 4)
    return fail(nullptr, DGMG_EINVAL, "problem too large");
  sp.P = o->P;
  sp.flux = o->flux;
  for (int d = 0; d < 3; ++d) sp.beta[d] = o->beta[d];
  sp.mu_star = o->mu_star;
  sp.smoother = o->smoother;
  sp.overlap = o->overlap;
  sp.weighting = o->weighting;
  dgmg_handle* h = new dgmg_handle();
  h->sp = sp;
  h->opts = *o;
  std::string e = build_levels(sp, h->lv);
  if (!e.empty()) {
    delete h;
    return fail(nullptr, DGMG_EINVAL, e);
  }
  // kernels must exist for every smoothing level
  for (size_t l = 1; l < h->lv.size(); ++l) {
    const LevelHost& lv = h->lv[l];
    const int NL = lv.NP + 2 * lv.NO;
    bool ok = o->smoother == DGMG_SMOOTHER_EA
                  ? (g->dim == 3 ? Kern<double, 3>::fdm_supported(NL, NL) : Kern<double, 2>::fdm_supported(NL, NL))
                  : (g->dim == 3 ? Kern<double, 3>::fdm_supported(2 * lv.P, NL) : Kern<double, 2>::fdm_supported(2 * lv.P, NL));
    if (!ok) {
      delete h;
      return fail(nullptr, DGMG_EUNSUPPORTED, "no patch kernel for P_l=" + std::to_string(lv.P) + " N_O=" + std::to_string(lv.NO));
    }
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
  h->stream = (hipStream_t)stream;
  h->ws = (char*)dev;
  h->ws_bytes = bytes;
  std::vector<std::pair<void*, std::vector<char>>> up;
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
  h->stream = (hipStream_t)stream;
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
  hipLaunchKernelGGL(k_mass, dim3((unsigned)((L.n_dof + 255) / 256)), dim3(256), 0, h->stream, L, f, g);
  return check_hip(h, "mass");
}

int dgmg_solve(dgmg_handle* h, const double* rhs, double* x, double tol, dgmg_stats* st) {
  int rc = need_bound(h);
  if (rc) return rc;
  if (!rhs || !x || !(tol >= 0)) return fail(h, DGMG_EINVAL, "bad arguments");
  const int L = (int)h->lv.size() - 1;
  const int64_t n = h->lv[L].n_dof;
  double* r = h->pr;
  double* ro = h->pro;
  double* p = h->pp;
  double* q = h->pq;
  double* z = h->pz;
  double* part1 = h->part;
  double* part2 = h->part + std::max<size_t>(2 * RED_BLOCKS, h->lv.back().n_elem + 8);
  double* S = h->scal;  // slots: 0,1 delta (alternating), 2 pq, 3 rr, 4 zdr, 5 zr
  const dim3 vb(RED_BLOCKS), vt(VEC_THREADS);
  if (st) std::memset(st, 0, sizeof(*st));
  // r = g - A x ; r_old = 0
  rc = k_apply<double>(h, L, 1, x, rhs, r, nullptr, nullptr);
  if (rc) return rc;
  k_fill_v<double>(h, ro, n);
  hipLaunchKernelGGL(k_dot, vb, vt, 0, h->stream, r, r, n, part1);
  hipLaunchKernelGGL(k_finalize, dim3(1), vt, 0, h->stream, part1, RED_BLOCKS, S + 3);
  double rr;
  if ((rc = read_scalar(h, S + 3, &rr))) return rc;
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
  // p = MG(r); delta = p.r
  if ((rc = precond(h, r, p))) return rc;
  hipLaunchKernelGGL(k_dot, vb, vt, 0, h->stream, p, r, n, part1);
  hipLaunchKernelGGL(k_finalize, dim3(1), vt, 0, h->stream, part1, RED_BLOCKS, S + 0);
  int cur = 0;
  int it = 0;
  double rn = r0;
  for (it = 1; it <= h->opts.max_iter; ++it) {
    int nb = 0;
    // q = A p, partial p.q
    rc = k_apply<double>(h, L, 2, p, nullptr, q, part1, &nb);
    if (rc) return rc;
    hipLaunchKernelGGL(k_finalize, dim3(1), vt, 0, h->stream, part1, nb, S + 2);
    hipLaunchKernelGGL(k_update_xr, vb, vt, 0, h->stream, x, r, p, q, S + cur, S + 2, n, part2);
    hipLaunchKernelGGL(k_finalize, dim3(1), vt, 0, h->stream, part2, RED_BLOCKS, S + 3);
    if ((rc = check_hip(h, "pcg update"))) return rc;
    if ((rc = read_scalar(h, S + 3, &rr))) return rc;
    rn = std::sqrt(rr);
    if (st) {
      st->iterations = it;
      st->r_final = rn;
      if (it < 256) st->history[it] = rn;
    }
    if (!std::isfinite(rn)) return fail(h, DGMG_ENONFINITE, "residual norm is not finite");
    if (rn <= rmax) break;
    if ((rc = precond(h, r, z))) return rc;
    hipLaunchKernelGGL(k_dot_zr, vb, vt, 0, h->stream, z, r, ro, n, part1, part2);
    hipLaunchKernelGGL(k_finalize, dim3(1), vt, 0, h->stream, part1, RED_BLOCKS, S + 4);
    hipLaunchKernelGGL(k_finalize, dim3(1), vt, 0, h->stream, part2, RED_BLOCKS, S + (cur ^ 1));
    hipLaunchKernelGGL(k_update_p, vb, vt, 0, h->stream, p, z, r, ro, S + 4, S + cur, n);
    cur ^= 1;
  }
  if ((rc = check_hip(h, "pcg"))) return rc;
  const bool conv = rn <= rmax;
  if (st) {
    st->converged = conv;
    if (st->iterations > 0) st->rho = std::pow(rn / r0, 1.0 / st->iterations);
  }
  return conv ? DGMG_OK : DGMG_NOT_CONVERGED;
}

int dgmg_kernel_timing(dgmg_handle* h, int enable) {
  if (!h) return DGMG_EINVAL;
  for (auto& e : h->ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  h->ev.clear();
  h->ev_flops.clear();
  h->ev_bytes.clear();
  h->t_ms = h->t_flops = h->t_bytes = 0;
  h->t_launch = 0;
  h->timing = enable != 0;
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
    (void)hipEventDestroy(h->ev[i].first);
    (void)hipEventDestroy(h->ev[i].second);
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
  if (h->host_scal) (void)hipHostFree(h->host_scal);
  delete h;
}

const char* dgmg_last_error(const dgmg_handle* h) {
  return h ? h->err.c_str() : g_setup_error.c_str();
}

}  // extern "C"

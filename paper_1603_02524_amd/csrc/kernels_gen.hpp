// Kernels for orders without compiled instances (P_l outside 1, 2, 3, 4, 6,
// 8, 12, 16, 32): the same operations as kernels.hpp with the order and the
// patch tile known only at run time.  Plain VALU loops, one thread per node
// (operator, overlap sum) or per line (patch solve); correct for every order
// whose tiles fit the LDS, but without the tuned data paths of the compiled
// kernels.  Same vector layouts, patch-buffer layout and summation orders of
// the overlap sum as the compiled kernels.
#pragma once

#include "kernels.hpp"

namespace dgmg {

constexpr int GEN_MAXLEN = 64;  // longest 1D line of a run-time tile (2 P for P <= 32)

// Element, local node and per-direction coordinates of node q (element-major).
struct GenNode {
  int e, loc, i[3], m[3];
};
template <class T>
__device__ __forceinline__ GenNode gen_node(const LevelDev<T>& L, int64_t q) {
  GenNode g;
  const int NP = L.NP, dim = L.dim;
  const int NE = dim == 3 ? NP * NP * NP : NP * NP;
  g.e = (int)(q / NE);
  g.loc = (int)(q - (int64_t)g.e * NE);
  g.i[0] = g.loc % NP;
  g.i[1] = (g.loc / NP) % NP;
  g.i[2] = dim == 3 ? g.loc / (NP * NP) : 0;
  const int N1 = L.dir[0].N, N2 = L.dir[1].N;
  g.m[0] = g.e % N1;
  g.m[1] = dim == 3 ? (g.e / N1) % N2 : g.e / N1;
  g.m[2] = dim == 3 ? g.e / (N1 * N2) : 0;
  return g;
}

// y = A x (MODE 0) or y = f - A x (MODE 1), eq. (L:generic) per direction:
// the element's own block (stiffness, face consistency and penalty terms) and
// the left / right neighbour blocks, times the other directions' masses.
template <class T>
__global__ void __launch_bounds__(256) gen_apply_kernel(LevelDev<T> L, int mode, const T* __restrict__ x,
                                                        const T* __restrict__ f, T* __restrict__ y) {
  if (inactive(L.active)) return;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.n_dof) return;
  const int NP = L.NP, P = NP - 1, dim = L.dim;
  const int NE = dim == 3 ? NP * NP * NP : NP * NP;
  const GenNode g = gen_node(L, q);
  const T* __restrict__ Ls = L.Ls;
  const T* __restrict__ D0 = L.D;
  const T* __restrict__ DP = L.D + P * NP;
  T acc = T(0);
  for (int d = 0; d < dim; ++d) {
    const DirDev<T>& dd = L.dir[d];
    const int i = g.i[d], md = g.m[d];
    const int sd = d == 0 ? 1 : (d == 1 ? NP : NP * NP);
    const int64_t est = d == 0 ? 1 : (d == 1 ? (int64_t)L.dir[0].N : (int64_t)L.dir[0].N * L.dir[1].N);
    const int base = g.loc - i * sd;
    const T* c = dd.ecoef + md * ECOEF_N;
    const T* xl = x + (int64_t)g.e * NE + base;
    T sL = T(0), s0 = T(0), sP = T(0);
    for (int k = 0; k < NP; ++k) {
      const T v = xl[k * sd];
      sL += Ls[i * NP + k] * v;
      s0 += D0[k] * v;
      sP += DP[k] * v;
    }
    T s = c[E_TWO_DX] * sL;
    s += c[E_CL] * (D0[i] * xl[0] + (i == 0 ? s0 : T(0)));
    if (i == 0) s += c[E_BL] * xl[0];
    s -= c[E_CR] * (DP[i] * xl[P * sd] + (i == P ? sP : T(0)));
    if (i == P) s += c[E_BR] * xl[P * sd];
    const int ml = dd.nbr[2 * md], mr = dd.nbr[2 * md + 1];
    if (ml >= 0) {
      const T* xn = x + ((int64_t)g.e + (int64_t)(ml - md) * est) * NE + base;
      T t = T(0);
      if (i == 0)
        for (int k = 0; k < NP; ++k) t += DP[k] * xn[k * sd];
      s += (-c[E_CL] * D0[i] - (i == 0 ? c[E_BL] : T(0))) * xn[P * sd] + (i == 0 ? c[E_CNL] * t : T(0));
    }
    if (mr >= 0) {
      const T* xn = x + ((int64_t)g.e + (int64_t)(mr - md) * est) * NE + base;
      T t = T(0);
      if (i == P)
        for (int k = 0; k < NP; ++k) t += D0[k] * xn[k * sd];
      s += (c[E_CR] * DP[i] - (i == P ? c[E_BR] : T(0))) * xn[0] - (i == P ? c[E_CNR] * t : T(0));
    }
    T mass = T(1);
    for (int d2 = 0; d2 < dim; ++d2)
      if (d2 != d) mass *= L.dir[d2].ecoef[g.m[d2] * ECOEF_N + E_HALF_DX] * L.rho[g.i[d2]];
    acc += mass * s;
  }
  y[q] = mode == 1 ? f[q] - acc : acc;
}

// Patch solve of one sweep (ND = nd, -1 element-centred) for a run-time tile:
// the same gather, fast-diagonalisation passes, eigenvalue scaling, weights and
// output layout (tile in grid-natural order, one tile per patch) as fdm_kernel.
// One LDS tile; a pass gives each thread whole lines (the line's results in a
// private buffer until all its inputs are read).
template <class T>
__global__ void __launch_bounds__(256) gen_fdm_kernel(LevelDev<T> L, int nd, int NA, int NL, const T* __restrict__ r,
                                                      T* __restrict__ out, int npx, int npy, int npz, PatchLat lat) {
  extern __shared__ __align__(16) unsigned char gen_smem[];
  T* tile = reinterpret_cast<T*>(gen_smem);
  const int dim = L.dim;
  const int pid = xcd_block(npx * npy * (dim == 3 ? npz : 1));
  if (pid < 0 || inactive(L.active)) return;
  int p[3];
  p[0] = lat.start[0] + lat.stride[0] * (pid % npx);
  p[1] = lat.start[1] + lat.stride[1] * ((pid / npx) % npy);
  p[2] = dim == 3 ? lat.start[2] + lat.stride[2] * (pid / (npx * npy)) : 0;
  int len[3] = {1, 1, 1};
  const int *go[3] = {nullptr, nullptr, nullptr};
  const T *wg[3] = {nullptr, nullptr, nullptr}, *lam[3] = {nullptr, nullptr, nullptr}, *S[3] = {nullptr, nullptr, nullptr};
  for (int d = 0; d < dim; ++d) {
    const DirDev<T>& dd = L.dir[d];
    const bool fc = d == nd;
    len[d] = fc ? NA : NL;
    go[d] = fc ? dd.goff_fc + p[d] * NA : dd.goff_ec + p[d] * NL;
    wg[d] = fc ? dd.w_fc + p[d] * NA : dd.w_ec + p[d] * NL;
    lam[d] = fc ? dd.lam_fc + p[d] * NA : dd.lam_ec + p[d] * NL;
    S[d] = fc ? dd.S_fc + (int64_t)p[d] * NA * NA : dd.S_ec + (int64_t)p[d] * NL * NL;
  }
  const int TS = len[0] * len[1] * len[2];
  const int st[3] = {1, len[0], len[0] * len[1]};
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int q = tid; q < TS; q += nth) {
    const int o0 = q % len[0], o1 = (q / len[0]) % len[1], o2 = q / (len[0] * len[1]);
    const int g0 = go[0][o0], g1 = go[1][o1], g2 = dim == 3 ? go[2][o2] : 0;
    tile[q] = (g0 | g1 | g2) < 0 ? T(0) : r[g0 + g1 + g2];
  }
  __syncthreads();
  // fwd (forward: t_j = sum_k S_kj v_k) for d = 0 .. dim-1, scale, then backward
  // (u_k = sum_j S_kj t_j) for d = dim-1 .. 0
  for (int step = 0; step < 2 * dim; ++step) {
    const bool fwd = step < dim;
    const int d = fwd ? step : 2 * dim - 1 - step;
    const int n = len[d], sd = st[d], lines = TS / n;
    const T* __restrict__ Sd = S[d];
    for (int ln = tid; ln < lines; ln += nth) {
      // line ln: the tile positions with coordinate d running, the others fixed
      const int lo = ln % sd, hi = ln / sd;
      const int base = lo + hi * sd * n;
      T res[GEN_MAXLEN];
      for (int j = 0; j < n; ++j) {
        T s = T(0);
        for (int k = 0; k < n; ++k) s += (fwd ? Sd[k * n + j] : Sd[j * n + k]) * tile[base + k * sd];
        res[j] = s;
      }
      for (int j = 0; j < n; ++j) tile[base + j * sd] = res[j];
    }
    __syncthreads();
    if (step == dim - 1) {
      for (int q = tid; q < TS; q += nth) {
        const int o0 = q % len[0], o1 = (q / len[0]) % len[1], o2 = q / (len[0] * len[1]);
        T den = lam[0][o0] + lam[1][o1];
        if (dim == 3) den += lam[2][o2];
        tile[q] = tile[q] / den;
      }
      __syncthreads();
    }
  }
  T* dst = out + (int64_t)pid * TS;
  for (int q = tid; q < TS; q += nth) {
    const int o0 = q % len[0], o1 = (q / len[0]) % len[1], o2 = q / (len[0] * len[1]);
    T w = wg[0][o0] * wg[1][o1];
    if (dim == 3) w *= wg[2][o2];
    dst[q] = w * tile[q];
  }
}

// u (+)= the overlap sum per node, as combine_kernel: per direction the
// candidate patches (face-centred along nd: faces m and m + 1; element-centred:
// patches m - 1, m, m + 1 within N_O), summed in the order z, y, x candidates.
template <class T>
__global__ void __launch_bounds__(256) gen_combine_kernel(LevelDev<T> L, int nd, int NA, int NL,
                                                          const T* __restrict__ buf, T* __restrict__ u, int npx,
                                                          int npy, int assign) {
  if (inactive(L.active)) return;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.n_dof) return;
  const int NP = L.NP, P = NP - 1, NO = L.NO, dim = L.dim;
  const GenNode g = gen_node(L, q);
  int len[3] = {1, 1, 1};
  for (int d = 0; d < dim; ++d) len[d] = d == nd ? NA : NL;
  const int64_t TS = (int64_t)len[0] * len[1] * len[2];
  const int64_t pst[3] = {1, npx, (int64_t)npx * npy};
  const int64_t ost[3] = {1, len[0], (int64_t)len[0] * len[1]};
  int cnt[3] = {1, 1, 1};
  int64_t adr[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int d = 0; d < dim; ++d) {
    const DirDev<T>& dd = L.dir[d];
    const int N = dd.N, md = g.m[d], i = g.i[d];
    int c = 0;
    if (d == nd) {
      if (i < P) adr[d][c++] = md * pst[d] * TS + (P + i) * ost[d];
      if (i >= 1) adr[d][c++] = (dd.periodic ? (md + 1) % N : md + 1) * pst[d] * TS + (i - 1) * ost[d];
    } else {
      if (i < NO && (dd.periodic || md > 0)) adr[d][c++] = ((md - 1 + N) % N) * pst[d] * TS + (NP + NO + i) * ost[d];
      adr[d][c++] = md * pst[d] * TS + (i + NO) * ost[d];
      if (i >= NP - NO && (dd.periodic || md < N - 1)) adr[d][c++] = ((md + 1) % N) * pst[d] * TS + (i - NP + NO) * ost[d];
    }
    cnt[d] = c;
  }
  T s = T(0);
  for (int c = 0; c < cnt[2]; ++c)
    for (int b = 0; b < cnt[1]; ++b)
      for (int a = 0; a < cnt[0]; ++a) s += buf[adr[0][a] + adr[1][b] + adr[2][c]];
  u[q] = assign ? s : u[q] + s;
}

// Element-local transfers with J (NPF x NPC): RESTRICT out_c = (J^T)^(x D) in_f,
// else out_f += J^(x D) in_c.  One block per element; two LDS buffers of
// NPF^D values; one pass per direction.
template <class T>
__global__ void __launch_bounds__(256) gen_transfer_kernel(LevelDev<T> Lf, int restrict_, const T* __restrict__ in,
                                                           T* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char gen_smem[];
  const int dim = Lf.dim, NPF = Lf.NP, NPC = Lf.NPc;
  const int NEF = dim == 3 ? NPF * NPF * NPF : NPF * NPF;
  const int NEC = dim == 3 ? NPC * NPC * NPC : NPC * NPC;
  T* a = reinterpret_cast<T*>(gen_smem);
  T* b = a + NEF;
  const int e = xcd_block(Lf.n_elem);
  if (e < 0 || inactive(Lf.active)) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int NIN = restrict_ ? NPF : NPC, NOUT = restrict_ ? NPC : NPF;
  const int nin = restrict_ ? NEF : NEC;
  for (int q = tid; q < nin; q += nth) a[q] = in[(int64_t)e * nin + q];
  __syncthreads();
  int ext[3] = {NIN, NIN, dim == 3 ? NIN : 1};
  T* src = a;
  T* dst = b;
  for (int d = 0; d < dim; ++d) {
    int oext[3] = {ext[0], ext[1], ext[2]};
    oext[d] = NOUT;
    const int no = oext[0] * oext[1] * oext[2];
    const int sin = d == 0 ? 1 : (d == 1 ? ext[0] : ext[0] * ext[1]);
    for (int q = tid; q < no; q += nth) {
      int o[3] = {q % oext[0], (q / oext[0]) % oext[1], q / (oext[0] * oext[1])};
      const int io = o[d];
      o[d] = 0;
      const int base = o[0] + o[1] * ext[0] + o[2] * ext[0] * ext[1];
      T s = T(0);
      for (int k = 0; k < NIN; ++k)
        s += (restrict_ ? Lf.J[k * NPC + io] : Lf.J[io * NPC + k]) * src[base + k * sin];
      dst[q] = s;
    }
    __syncthreads();
    ext[d] = NOUT;
    T* t = src;
    src = dst;
    dst = t;
  }
  const int nout = restrict_ ? NEC : NEF;
  for (int q = tid; q < nout; q += nth) {
    if (restrict_) out[(int64_t)e * NEC + q] = src[q];
    else out[(int64_t)e * NEF + q] += src[q];
  }
}

// ------------------------------------------------------------------ launchers
inline unsigned gen_node_blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

template <class T>
size_t gen_fdm_shmem(int dim, int NA, int NL) {
  return (size_t)NA * NL * (dim == 3 ? NL : 1) * sizeof(T);
}
// the run-time patch solve fits: one tile in LDS and lines of at most GEN_MAXLEN
template <class T>
bool gen_fdm_fits(int dim, int NA, int NL) {
  return NA <= GEN_MAXLEN && NL <= GEN_MAXLEN && gen_fdm_shmem<T>(dim, NA, NL) <= 160 * 1024;
}
template <class T>
size_t gen_transfer_shmem(int dim, int NPF) {
  return 2 * (size_t)NPF * NPF * (dim == 3 ? NPF : 1) * sizeof(T);
}

template <class T>
int gen_apply_launch(const LevelDev<T>& L, int mode, const T* x, const T* f, T* y, hipStream_t s) {
  if (mode != 0 && mode != 1) return -4;
  hipLaunchKernelGGL((gen_apply_kernel<T>), dim3(gen_node_blocks(L.n_dof)), dim3(256), 0, s, L, mode, x, f, y);
  return 0;
}

template <class T>
int gen_fdm_launch(const LevelDev<T>& L, int nd, int NA, int NL, const T* r, T* out, int npx, int npy, int npz,
                   const PatchLat& lat, hipStream_t s) {
  if (!gen_fdm_fits<T>(L.dim, NA, NL)) return -4;
  const size_t shm = gen_fdm_shmem<T>(L.dim, NA, NL);
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)gen_fdm_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  const int np = npx * npy * (L.dim == 3 ? npz : 1);
  hipLaunchKernelGGL((gen_fdm_kernel<T>), dim3(xcd_grid(np)), dim3(256), shm, s, L, nd, NA, NL, r, out, npx, npy, npz,
                     lat);
  return 0;
}

template <class T>
int gen_combine_launch(const LevelDev<T>& L, int nd, int NA, int NL, const T* buf, T* u, int npx, int npy,
                       bool assign, hipStream_t s) {
  hipLaunchKernelGGL((gen_combine_kernel<T>), dim3(gen_node_blocks(L.n_dof)), dim3(256), 0, s, L, nd, NA, NL, buf, u,
                     npx, npy, assign ? 1 : 0);
  return 0;
}

template <class T>
int gen_transfer_launch(const LevelDev<T>& Lf, bool restrict_, const T* in, T* out, hipStream_t s) {
  const size_t shm = gen_transfer_shmem<T>(Lf.dim, Lf.NP);
  if (shm > 160 * 1024) return -4;
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)gen_transfer_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)shm);
  hipLaunchKernelGGL((gen_transfer_kernel<T>), dim3(xcd_grid(Lf.n_elem)), dim3(256), shm, s, Lf, restrict_ ? 1 : 0,
                     in, out);
  return 0;
}

}  // namespace dgmg

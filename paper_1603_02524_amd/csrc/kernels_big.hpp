// Kernels for 3D levels whose element or patch tiles exceed the LDS of one
// workgroup (N_P = 33 at P = 32: an element holds 33^3 nodes, a face-centred
// patch 64 x 43 x 43).  Same operations and layouts as kernels.hpp; the data
// that do not fit are kept in global memory (L2 / MALL resident) between
// passes instead of LDS.
#pragma once

#include "kernels.hpp"

namespace dgmg {

constexpr int BIG_NP = 33;  // N_P of the largest order (P = 32)

// ================================================================ operator apply
// One block per element.  For each direction every thread owns lines of that
// direction (as in apply_kernel); the partial sums over the directions live in
// y itself, which only this block touches, and the barrier between directions
// orders them: y = A x (MODE 0), y = f - A x accumulated as ((f - c0) - c1) - c2
// so that y may alias f (MODE 1), y = A x with the block's x.y partial (MODE 2).
// y must not alias x.
template <class T, int NP, int MODE>
__global__ void __launch_bounds__(256) apply_big_kernel(LevelDev<T> L, const T* __restrict__ x, const T* f,
                                                        T* y, double* __restrict__ part, int nblk) {
  constexpr int NE = NP * NP * NP, NLN = NP * NP, P = NP - 1;
  __shared__ double red[16];
  __shared__ T sLs[NP * NP], sD0[NP], sDP[NP], srho[NP];
  const int e = xcd_block(nblk);
  if (e < 0 || inactive(L.active)) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int q = tid; q < NP * NP; q += nth) sLs[q] = L.Ls[q];
  for (int q = tid; q < NP; q += nth) {
    sD0[q] = L.D[q];
    sDP[q] = L.D[P * NP + q];
    srho[q] = L.rho[q];
  }
  __syncthreads();
  const int N1 = L.dir[0].N, N2 = L.dir[1].N;
  int m[3];
  m[0] = e % N1;
  m[1] = (e / N1) % N2;
  m[2] = e / (N1 * N2);
  const int64_t g0 = (int64_t)e * NE;
  double acc = 0.0;
#pragma unroll 1
  for (int d = 0; d < 3; ++d) {
    const DirDev<T> dd = L.dir[d];
    const int estride = d == 0 ? 1 : (d == 1 ? N1 : N1 * N2);
    const T* c = dd.ecoef + m[d] * ECOEF_N;
    const int nl = dd.nbr[2 * m[d]], nr = dd.nbr[2 * m[d] + 1];
    const int da = d == 0 ? 1 : 0, db = d == 2 ? 1 : 2;
    const T ha = L.dir[da].ecoef[m[da] * ECOEF_N + E_HALF_DX], hb = L.dir[db].ecoef[m[db] * ECOEF_N + E_HALF_DX];
    for (int t = tid; t < NLN; t += nth) {
      int base, stride;
      const int ia = t % NP, ib = t / NP;
      if (d == 0) {
        base = t * NP; stride = 1;
      } else if (d == 1) {
        base = ia + ib * NP * NP; stride = NP;
      } else {
        base = t; stride = NP * NP;
      }
      T v[NP];
#pragma unroll
      for (int k = 0; k < NP; ++k) v[k] = x[g0 + base + k * stride];
      T d0 = 0, dP = 0;
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        d0 += sD0[k] * v[k];
        dP += sDP[k] * v[k];
      }
      T uL = 0, dL = 0, uR = 0, dR = 0;
      if (nl >= 0) {
        const T* w = x + (int64_t)(e + (nl - m[d]) * estride) * NE + base;
#pragma unroll
        for (int k = 0; k < NP; ++k) dL += sDP[k] * w[k * stride];
        uL = w[P * stride];
      }
      if (nr >= 0) {
        const T* w = x + (int64_t)(e + (nr - m[d]) * estride) * NE + base;
#pragma unroll
        for (int k = 0; k < NP; ++k) dR += sD0[k] * w[k * stride];
        uR = w[0];
      }
      const T jl = v[0] - uL, jr = v[P] - uR;
      const T fl = c[E_CL] * d0 + c[E_CNL] * dL + c[E_BL] * jl;
      const T fr = -c[E_CR] * dP - c[E_CNR] * dR + c[E_BR] * jr;
      const T cl = c[E_CL] * jl, cr = c[E_CR] * jr, tdx = c[E_TWO_DX];
      const T mo = ha * srho[ia] * hb * srho[ib];
      for (int i = 0; i < NP; ++i) {
        T s = 0;
#pragma unroll
        for (int k = 0; k < NP; ++k) s += sLs[i * NP + k] * v[k];
        T o = tdx * s + cl * sD0[i] - cr * sDP[i];
        if (i == 0) o += fl;
        if (i == P) o += fr;
        const int64_t idx = g0 + base + i * stride;
        const T val = mo * o;
        if (MODE == 1) {
          y[idx] = (d == 0 ? f[idx] : y[idx]) - val;
        } else if (d == 0) {
          y[idx] = val;
        } else {
          const T tot = y[idx] + val;
          y[idx] = tot;
          if (MODE == 2 && d == 2) acc += (double)v[i] * (double)tot;
        }
      }
    }
    __syncthreads();
  }
  if (MODE == 2) {
    const double s = block_sum(acc, red);
    if (tid == 0) part[e] = s;
  }
}

template <class T, int NP>
int apply_big_launch(const LevelDev<T>& L, int mode, const T* x, const T* f, T* y, double* part, int* nblk_out,
                     hipStream_t s) {
  const int nblk = L.n_elem;
  if (nblk_out) *nblk_out = nblk;
  dim3 grid(xcd_grid(nblk)), block(256);
  if (mode == 0)
    hipLaunchKernelGGL((apply_big_kernel<T, NP, 0>), grid, block, 0, s, L, x, f, y, part, nblk);
  else if (mode == 1)
    hipLaunchKernelGGL((apply_big_kernel<T, NP, 1>), grid, block, 0, s, L, x, f, y, part, nblk);
  else
    hipLaunchKernelGGL((apply_big_kernel<T, NP, 2>), grid, block, 0, s, L, x, f, y, part, nblk);
  return 0;
}

// ================================================================ p-transfers
// Restriction out_c = (J^T x J^T x J^T) in_f in two kernels: the slowest
// direction through the scratch tmp [e][k'][j][i], then the two fast
// directions per (element, k') plane in LDS.  Prolongation out_f += (J x J x J)
// in_c: the two fast directions per coarse plane into tmp [e][k][j][i], then
// the slowest direction accumulated into out.
template <class T, int NPF, int NPC>
__global__ void __launch_bounds__(256) restrict_z_kernel(const T* __restrict__ J, int n_elem,
                                                         const T* __restrict__ in, T* __restrict__ tmp,
                                                         const int* __restrict__ active) {
  if (inactive(active)) return;
  constexpr int PL = NPF * NPF, NEF = NPF * PL, PER = NPC * PL;
  const int64_t total = (int64_t)n_elem * PER;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = q / PER;
    const int r = (int)(q - e * PER), kc = r / PL, ji = r - kc * PL;
    const T* src = in + e * NEF + ji;
    T s = 0;
#pragma unroll
    for (int k = 0; k < NPF; ++k) s += J[k * NPC + kc] * src[k * PL];
    tmp[q] = s;
  }
}

template <class T, int NPF, int NPC>
__global__ void __launch_bounds__(256) restrict_xy_kernel(const T* __restrict__ J, int n_elem,
                                                          const T* __restrict__ tmp, T* __restrict__ out,
                                                          const int* __restrict__ active) {
  if (inactive(active)) return;
  constexpr int PL = NPF * NPF, NEC = NPC * NPC * NPC;
  __shared__ T pl[PL], t1[NPF * NPC], sJ[NPF * NPC];
  const int64_t b = blockIdx.x;
  const int64_t e = b / NPC;
  const int kc = (int)(b - e * NPC);
  if (e >= n_elem) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  const T* src = tmp + b * PL;
  for (int q = tid; q < PL; q += nth) pl[q] = src[q];
  for (int q = tid; q < NPF * NPC; q += nth) sJ[q] = J[q];
  __syncthreads();
  for (int q = tid; q < NPF * NPC; q += nth) {  // t1[j][i'] = sum_i J[i][i'] pl[j][i]
    const int j = q / NPC, ic = q - j * NPC;
    T s = 0;
    for (int i = 0; i < NPF; ++i) s += sJ[i * NPC + ic] * pl[j * NPF + i];
    t1[q] = s;
  }
  __syncthreads();
  T* dst = out + e * NEC + (int64_t)kc * NPC * NPC;
  for (int q = tid; q < NPC * NPC; q += nth) {  // out[j'][i'] = sum_j J[j][j'] t1[j][i']
    const int jc = q / NPC, ic = q - jc * NPC;
    T s = 0;
    for (int j = 0; j < NPF; ++j) s += sJ[j * NPC + jc] * t1[j * NPC + ic];
    dst[q] = s;
  }
}

template <class T, int NPF, int NPC>
__global__ void __launch_bounds__(256) prolong_xy_kernel(const T* __restrict__ J, int n_elem,
                                                         const T* __restrict__ in, T* __restrict__ tmp,
                                                         const int* __restrict__ active) {
  if (inactive(active)) return;
  constexpr int PLF = NPF * NPF, NEC = NPC * NPC * NPC;
  __shared__ T pl[NPC * NPC], t1[NPC * NPF], sJ[NPF * NPC];
  const int64_t b = blockIdx.x;
  const int64_t e = b / NPC;
  const int kc = (int)(b - e * NPC);
  if (e >= n_elem) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  const T* src = in + e * NEC + (int64_t)kc * NPC * NPC;
  for (int q = tid; q < NPC * NPC; q += nth) pl[q] = src[q];
  for (int q = tid; q < NPF * NPC; q += nth) sJ[q] = J[q];
  __syncthreads();
  for (int q = tid; q < NPC * NPF; q += nth) {  // t1[j'][i] = sum_i' J[i][i'] pl[j'][i']
    const int jc = q / NPF, i = q - jc * NPF;
    T s = 0;
    for (int ic = 0; ic < NPC; ++ic) s += sJ[i * NPC + ic] * pl[jc * NPC + ic];
    t1[q] = s;
  }
  __syncthreads();
  T* dst = tmp + b * PLF;
  for (int q = tid; q < PLF; q += nth) {  // tmp[j][i] = sum_j' J[j][j'] t1[j'][i]
    const int j = q / NPF, i = q - j * NPF;
    T s = 0;
    for (int jc = 0; jc < NPC; ++jc) s += sJ[j * NPC + jc] * t1[jc * NPF + i];
    dst[q] = s;
  }
}

template <class T, int NPF, int NPC>
__global__ void __launch_bounds__(256) prolong_z_kernel(const T* __restrict__ J, int n_elem,
                                                        const T* __restrict__ tmp, T* __restrict__ out,
                                                        const int* __restrict__ active) {
  if (inactive(active)) return;
  constexpr int PL = NPF * NPF, NEF = NPF * PL, TPE = NPC * PL;
  const int64_t total = (int64_t)n_elem * NEF;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = q / NEF;
    const int r = (int)(q - e * NEF), k = r / PL, ji = r - k * PL;
    const T* src = tmp + e * TPE + ji;
    T s = 0;
#pragma unroll
    for (int kc = 0; kc < NPC; ++kc) s += J[k * NPC + kc] * src[kc * PL];
    out[q] += s;
  }
}

// Scratch elements the two-kernel transfer needs (n_elem NPC NPF^2).
inline int64_t transfer_big_scratch(int n_elem, int NPF, int NPC) { return (int64_t)n_elem * NPC * NPF * NPF; }

template <class T, int NPF, int NPC>
int transfer_big_launch(const T* J, int n_elem, bool restrict_, const T* in, T* out, T* tmp, const int* active,
                        hipStream_t s) {
  const int64_t nz = (int64_t)n_elem * NPC * NPF * NPF;
  const unsigned gz = (unsigned)imin(65536, (int)((nz + 255) / 256));
  const unsigned gp = (unsigned)(n_elem * NPC);
  if (restrict_) {
    hipLaunchKernelGGL((restrict_z_kernel<T, NPF, NPC>), dim3(gz), dim3(256), 0, s, J, n_elem, in, tmp, active);
    hipLaunchKernelGGL((restrict_xy_kernel<T, NPF, NPC>), dim3(gp), dim3(256), 0, s, J, n_elem, tmp, out, active);
  } else {
    const int64_t nf = (int64_t)n_elem * NPF * NPF * NPF;
    const unsigned gf = (unsigned)imin(65536, (int)((nf + 255) / 256));
    hipLaunchKernelGGL((prolong_xy_kernel<T, NPF, NPC>), dim3(gp), dim3(256), 0, s, J, n_elem, in, tmp, active);
    hipLaunchKernelGGL((prolong_z_kernel<T, NPF, NPC>), dim3(gf), dim3(256), 0, s, J, n_elem, tmp, out, active);
  }
  return 0;
}

// ================================================================ FDM patch solve
// In-place line contraction on a 2D LDS array: for each of `lines` lines v
// (element k at tile[line * ls + k * ks]) out_j = sum_k B[k][j] v_k, B row-major
// LEN x LEN in global memory.  Lines are the M dimension of 16x16x4 matrix-core
// products (see Mfma), each wave owning whole blocks of 16 lines.
template <class T, int LEN>
__device__ __forceinline__ void mfma_lines(T* __restrict__ tile, int lines, int ls, int ks_,
                                           const T* __restrict__ Bm) {
  constexpr int KS = (LEN + 3) / 4, NB = (LEN + 15) / 16;
  using M = Mfma<T>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int MB = (lines + 15) / 16;
  if (wave >= MB) return;
  T b[NB][KS];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + lk, j = nb * 16 + li;
      b[nb][ks] = (k < LEN && j < LEN) ? Bm[k * LEN + j] : T(0);
    }
  for (int mb = wave; mb < MB; mb += nw) {
    const int line = mb * 16 + li;
    const bool lv = line < lines;
    const int base = lv ? line * ls : 0;
    typename M::acc_t acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = typename M::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + lk;
      const T a = (lv && k < LEN) ? tile[base + k * ks_] : T(0);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = M::op(a, b[nb][ks], acc[nb]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int oline = mb * 16 + M::row(lk, r);
      if (oline < lines) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const int j = nb * 16 + li;
          if (j < LEN) tile[oline * ls + j * ks_] = acc[nb][r];
        }
      }
    }
  }
}

// Contraction of length n in {NA, NL} (the two tile lengths of a patch).
template <class T, int NA, int NL>
__device__ __forceinline__ void mfma_lines_n(int n, T* tile, int lines, int ls, int ks_, const T* Bm) {
  if (n == NA)
    mfma_lines<T, NA>(tile, lines, ls, ks_, Bm);
  else
    mfma_lines<T, NL>(tile, lines, ls, ks_, Bm);
}

// Per-patch geometry shared by the three stages: tile lengths per grid
// direction (len[nd] = NA, else NL), start index of the patch range and the
// 1D tables of each direction.
template <class T>
struct BigPatch {
  int p[3], len[3], start[3];
  const T* w[3];
  const T* lam[3];
  const T* S[3];
  const T* ST[3];
};

template <class T, int NA, int NL>
__device__ __forceinline__ BigPatch<T> big_patch(const LevelDev<T>& L, int nd, int pid, int npx, int npy) {
  BigPatch<T> q;
  q.p[0] = pid % npx;
  q.p[1] = (pid / npx) % npy;
  q.p[2] = pid / (npx * npy);
  const int NP = L.NP;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const DirDev<T>& dd = L.dir[d];
    const bool fc = d == nd;
    q.len[d] = fc ? NA : NL;
    q.start[d] = fc ? (q.p[d] - 1) * NP + 1 : q.p[d] * NP - L.NO;
    q.w[d] = fc ? dd.w_fc + q.p[d] * NA : dd.w_ec + q.p[d] * NL;
    q.lam[d] = fc ? dd.lam_fc + q.p[d] * NA : dd.lam_ec + q.p[d] * NL;
    q.S[d] = fc ? dd.S_fc + (int64_t)q.p[d] * NA * NA : dd.S_ec + (int64_t)q.p[d] * NL * NL;
    q.ST[d] = fc ? dd.ST_fc + (int64_t)q.p[d] * NA * NA : dd.ST_ec + (int64_t)q.p[d] * NL * NL;
  }
  return q;
}

// Global offset of patch position o in direction d, or -1 outside a Dirichlet domain.
template <class T>
__device__ __forceinline__ int64_t big_goff(const LevelDev<T>& L, const BigPatch<T>& q, int d, int o) {
  const DirDev<T>& dd = L.dir[d];
  const int NP = L.NP, G = dd.N * NP;
  int g = q.start[d] + o;
  if (dd.periodic) g = ((g % G) + G) % G;
  if (g < 0 || g >= G) return -1;
  const int64_t NE = (int64_t)NP * NP * NP;
  const int64_t est = d == 0 ? NE : (d == 1 ? (int64_t)L.dir[0].N * NE : (int64_t)L.dir[0].N * L.dir[1].N * NE);
  const int nst = d == 0 ? 1 : (d == 1 ? NP : NP * NP);
  const int mm = g / NP, ii = g - mm * NP;
  return mm * est + (int64_t)ii * nst;
}

constexpr int big_pitch(int n) { return n % 2 == 0 ? n + 1 : n; }

// Stage A: block per (patch, o2).  Gather the plane o2 of R_s r, forward
// transform along directions 0 and 1, store it in the patch's slot
// (grid-natural order (o2 len1 + o1) len0 + o0).
template <class T, int NA, int NL>
__global__ void __launch_bounds__(256) fdm_big_a(LevelDev<T> L, int nd, const T* __restrict__ r,
                                                 T* __restrict__ out, int npx, int npy, int npz) {
  constexpr int NM = imax(NA, NL), PM = big_pitch(NM);
  __shared__ T pl[NM * PM];
  __shared__ int64_t g0[NM], g1[NM];
  const int len2 = nd == 2 ? NA : NL;
  const int npatch = npx * npy * npz;
  const int bid = xcd_block(npatch * len2);
  if (bid < 0 || inactive(L.active)) return;
  const int pid = bid / len2, o2 = bid - pid * len2;
  const BigPatch<T> q = big_patch<T, NA, NL>(L, nd, pid, npx, npy);
  const int n0 = q.len[0], n1 = q.len[1], pitch = big_pitch(n0);
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int o = tid; o < n0; o += nth) g0[o] = big_goff(L, q, 0, o);
  for (int o = tid; o < n1; o += nth) g1[o] = big_goff(L, q, 1, o);
  const int64_t gz = big_goff(L, q, 2, o2);
  __syncthreads();
  for (int e = tid; e < n0 * n1; e += nth) {
    const int o1 = e / n0, o0 = e - o1 * n0;
    const bool ok = gz >= 0 && g0[o0] >= 0 && g1[o1] >= 0;
    pl[o1 * pitch + o0] = ok ? r[gz + g0[o0] + g1[o1]] : T(0);
  }
  __syncthreads();
  mfma_lines_n<T, NA, NL>(n0, pl, n1, pitch, 1, q.S[0]);  // rows: direction 0
  __syncthreads();
  mfma_lines_n<T, NA, NL>(n1, pl, n0, 1, pitch, q.S[1]);  // columns: direction 1
  __syncthreads();
  T* dst = out + (int64_t)pid * n0 * n1 * len2 + (int64_t)o2 * n0 * n1;
  for (int e = tid; e < n0 * n1; e += nth) {
    const int o1 = e / n0, o0 = e - o1 * n0;
    dst[e] = pl[o1 * pitch + o0];
  }
}

// Stage B: block per (patch, o1).  Along direction 2: forward transform, scale
// by 1 / (lam0 + lam1 + lam2), backward transform; in place in the slot.
template <class T, int NA, int NL>
__global__ void __launch_bounds__(256) fdm_big_b(LevelDev<T> L, int nd, T* __restrict__ out, int npx, int npy,
                                                 int npz) {
  constexpr int NM = imax(NA, NL), PM = big_pitch(NM);
  __shared__ T pl[NM * PM];
  __shared__ T l0[NM], l2[NM];
  const int len1 = nd == 1 ? NA : NL;
  const int npatch = npx * npy * npz;
  const int bid = xcd_block(npatch * len1);
  if (bid < 0 || inactive(L.active)) return;
  const int pid = bid / len1, o1 = bid - pid * len1;
  const BigPatch<T> q = big_patch<T, NA, NL>(L, nd, pid, npx, npy);
  const int n0 = q.len[0], n1 = q.len[1], n2 = q.len[2], pitch = big_pitch(n0);
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int o = tid; o < n0; o += nth) l0[o] = q.lam[0][o];
  for (int o = tid; o < n2; o += nth) l2[o] = q.lam[2][o];
  const T l1 = q.lam[1][o1];
  T* slot = out + (int64_t)pid * n0 * n1 * n2 + (int64_t)o1 * n0;
  const int64_t zst = (int64_t)n0 * n1;
  for (int e = tid; e < n0 * n2; e += nth) {
    const int o2 = e / n0, o0 = e - o2 * n0;
    pl[o2 * pitch + o0] = slot[o2 * zst + o0];
  }
  __syncthreads();
  mfma_lines_n<T, NA, NL>(n2, pl, n0, 1, pitch, q.S[2]);
  __syncthreads();
  for (int e = tid; e < n0 * n2; e += nth) {
    const int o2 = e / n0, o0 = e - o2 * n0;
    const int i = o2 * pitch + o0;
    pl[i] = pl[i] / (l0[o0] + l1 + l2[o2]);
  }
  __syncthreads();
  mfma_lines_n<T, NA, NL>(n2, pl, n0, 1, pitch, q.ST[2]);
  __syncthreads();
  for (int e = tid; e < n0 * n2; e += nth) {
    const int o2 = e / n0, o0 = e - o2 * n0;
    slot[o2 * zst + o0] = pl[o2 * pitch + o0];
  }
}

// Stage C: block per (patch, o2).  Backward transform along directions 1 and 0,
// multiply by the weights w0 w1 w2; in place in the slot.
template <class T, int NA, int NL>
__global__ void __launch_bounds__(256) fdm_big_c(LevelDev<T> L, int nd, T* __restrict__ out, int npx, int npy,
                                                 int npz) {
  constexpr int NM = imax(NA, NL), PM = big_pitch(NM);
  __shared__ T pl[NM * PM];
  __shared__ T w0[NM], w1[NM];
  const int len2 = nd == 2 ? NA : NL;
  const int npatch = npx * npy * npz;
  const int bid = xcd_block(npatch * len2);
  if (bid < 0 || inactive(L.active)) return;
  const int pid = bid / len2, o2 = bid - pid * len2;
  const BigPatch<T> q = big_patch<T, NA, NL>(L, nd, pid, npx, npy);
  const int n0 = q.len[0], n1 = q.len[1], pitch = big_pitch(n0);
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int o = tid; o < n0; o += nth) w0[o] = q.w[0][o];
  for (int o = tid; o < n1; o += nth) w1[o] = q.w[1][o];
  const T w2 = q.w[2][o2];
  T* slot = out + (int64_t)pid * n0 * n1 * len2 + (int64_t)o2 * n0 * n1;
  for (int e = tid; e < n0 * n1; e += nth) {
    const int o1 = e / n0, o0 = e - o1 * n0;
    pl[o1 * pitch + o0] = slot[e];
  }
  __syncthreads();
  mfma_lines_n<T, NA, NL>(n1, pl, n0, 1, pitch, q.ST[1]);
  __syncthreads();
  mfma_lines_n<T, NA, NL>(n0, pl, n1, pitch, 1, q.ST[0]);
  __syncthreads();
  for (int e = tid; e < n0 * n1; e += nth) {
    const int o1 = e / n0, o0 = e - o1 * n0;
    slot[e] = w0[o0] * w1[o1] * w2 * pl[o1 * pitch + o0];
  }
}

template <class T, int NA, int NL>
int fdm_big_launch(const LevelDev<T>& L, int nd, const T* r, T* out, int npx, int npy, int npz, hipStream_t s) {
  const int npatch = npx * npy * npz;
  const int len1 = nd == 1 ? NA : NL, len2 = nd == 2 ? NA : NL;
  hipLaunchKernelGGL((fdm_big_a<T, NA, NL>), dim3(xcd_grid(npatch * len2)), dim3(256), 0, s, L, nd, r, out, npx,
                     npy, npz);
  hipLaunchKernelGGL((fdm_big_b<T, NA, NL>), dim3(xcd_grid(npatch * len1)), dim3(256), 0, s, L, nd, out, npx,
                     npy, npz);
  hipLaunchKernelGGL((fdm_big_c<T, NA, NL>), dim3(xcd_grid(npatch * len2)), dim3(256), 0, s, L, nd, out, npx,
                     npy, npz);
  return 0;
}

}  // namespace dgmg

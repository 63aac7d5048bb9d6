// Continuous spectral-element (SE) counterpart (Sec. 4.3): kernels on the
// global node lattice.
//
// Vector layout: per direction d the lattice positions g = m P + i of element
// m's nodes (neighbours share g = m P); a homogeneous Dirichlet direction
// stores g = 1 .. N P - 1 at g - 1, a periodic one g mod N P; entries
// s0 + nl0 (s1 + nl1 s2), direction 1 fastest (nl_d = DirDev::nl).
//
// Operator (direct stiffness summation): y = sum_e Q_e^T A_e Q_e x in two
// launches, the element-local A_e x_e of every element into an element-major
// buffer (se_elem_kernel), then per lattice node the sum of the copies of the
// elements sharing it, in a fixed order (se_dss_kernel).  No atomics: the
// result does not depend on the launch order.
// Smoother: the element-centred patch solves are the DG ones (fdm_kernel with
// the continuous tables and lattice offsets); their weighted corrections are
// summed per lattice node by se_combine_kernel.
// Transfers: prolongation per element onto the nodes it owns (i_d < P in every
// direction: each lattice node has exactly one owner); restriction per element
// with the shared fine nodes weighted by 1 / (number of elements sharing them)
// into an element-major coarse buffer, then the coarse node sum.
#pragma once

#include "kernels.hpp"

namespace dgmg {

// Stored index of lattice position g in a direction with N elements of order P
// (-1: a dropped Dirichlet node).
__device__ __forceinline__ int se_stored(int g, int P, int N, int periodic) {
  const int G = N * P;
  if (periodic) {
    g %= G;
    return g < 0 ? g + G : g;
  }
  return (g >= 1 && g <= G - 1) ? g - 1 : -1;
}

// Elements per block of the element kernels: about 256 lines of one direction.
template <int NP, int DIM>
constexpr int se_epb() {
  return imax(1, 256 / ipow(NP, DIM - 1));
}

// Lattice strides of the directions of level L.
template <class T>
__device__ __forceinline__ void se_strides(const LevelDev<T>& L, int64_t st[3]) {
  st[0] = 1;
  st[1] = L.dir[0].nl;
  st[2] = (int64_t)L.dir[0].nl * L.dir[1].nl;
}

// Per element of the block and direction: the stored offset of each local node
// (-1: dropped) into the lattice vector of level L.
template <class T, int DIM, int NP, int EPB>
__device__ __forceinline__ void se_elem_offsets(const LevelDev<T>& L, int e0, int ne, int64_t (*off)[3][NP]) {
  int64_t st[3];
  se_strides(L, st);
  const int N1 = L.dir[0].N, N2 = L.dir[1].N, P = NP - 1;
  for (int q = threadIdx.x; q < ne * DIM * NP; q += blockDim.x) {
    const int el = q / (DIM * NP), rem = q - el * DIM * NP, d = rem / NP, i = rem - d * NP;
    const int e = e0 + el;
    const int md = d == 0 ? e % N1 : (d == 1 ? (DIM == 3 ? (e / N1) % N2 : e / N1) : e / (N1 * N2));
    const DirDev<T>& dd = L.dir[d];
    const int s = se_stored(md * P + i, P, dd.N, dd.periodic);
    off[el][d][i] = s < 0 ? -1 : s * st[d];
  }
  if (DIM == 2)
    for (int q = threadIdx.x; q < ne; q += blockDim.x) off[q][2][0] = 0;
}

// w_e = A_e x_e for every element (element-major output, NP^DIM per element):
// A_e = sum_d (x)_{d' != d} (dx_{d'}/2) diag(rho) (x) (2/dx_d) L^s.  The block's
// elements are staged in LDS; then one pass per direction with one thread per
// line of that direction: the line's NP values in registers, the rows of L^s
// as uniform (scalar) operands, the line's factor (2/dx_d) prod (dx_d'/2) rho
// applied once per output; the passes accumulate in a second LDS tile in
// direction order.
// PN (small levels, few lines per block): one thread per line and output
// instead of per line, so that short launches still have enough parallel work.
template <class T, int DIM, int NP, bool PN>
__global__ void __launch_bounds__(1024) se_elem_kernel(LevelDev<T> L, const T* __restrict__ x, T* __restrict__ w,
                                                       int nblk, int epb) {
  constexpr int NE = ipow(NP, DIM), NLN = ipow(NP, DIM - 1), EPB = se_epb<NP, DIM>();
  __shared__ T xs[EPB * NE];
  __shared__ T acc[EPB * NE];
  __shared__ T srho[NP];
  __shared__ int64_t off[EPB][3][NP];
  __shared__ T two[EPB][3], half[EPB][3];
  constexpr bool SLS = NP * sizeof(T) <= 72;  // rows fit the scalar registers
  __shared__ T sLs[SLS ? 1 : NP * NP];
  const int blk = xcd_block(nblk);
  if (blk < 0 || inactive(L.active)) return;
  const int e0 = blk * epb, ne = imin(imin(epb, EPB), L.n_elem - e0);
  const int tid = threadIdx.x, nth = blockDim.x;
  if constexpr (!SLS)
    for (int q = tid; q < NP * NP; q += nth) sLs[q] = L.Ls[q];
  for (int q = tid; q < NP; q += nth) srho[q] = L.rho[q];
  const int N1 = L.dir[0].N, N2 = L.dir[1].N;
  for (int q = tid; q < ne * 3; q += nth) {
    const int el = q / 3, d = q - el * 3, e = e0 + el;
    if (d >= DIM) {
      two[el][d] = T(0);
      half[el][d] = T(1);
      continue;
    }
    const int md = d == 0 ? e % N1 : (d == 1 ? (DIM == 3 ? (e / N1) % N2 : e / N1) : e / (N1 * N2));
    two[el][d] = L.dir[d].ecoef[md * ECOEF_N + E_TWO_DX];
    half[el][d] = L.dir[d].ecoef[md * ECOEF_N + E_HALF_DX];
  }
  se_elem_offsets<T, DIM, NP, EPB>(L, e0, ne, off);
  __syncthreads();
  // gather: GU loads of a thread in flight before their LDS stores
  constexpr int GU = 8;
  for (int q0 = tid; q0 < ne * NE; q0 += GU * nth) {
    T v[GU];
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int q = q0 + u * nth;
      const int qq = q < ne * NE ? q : 0;
      const int el = qq / NE, loc = qq - el * NE;
      const int i = loc % NP, j = (loc / NP) % NP, k = DIM == 3 ? loc / (NP * NP) : 0;
      const int64_t a = off[el][0][i], b = off[el][1][j], c = off[el][2][k];
      const bool ok = q < ne * NE && (a | b | c) >= 0;
      T t = T(0);
      if (ok) t = x[a + b + c];
      v[u] = t;
    }
#pragma unroll
    for (int u = 0; u < GU; ++u)
      if (q0 + u * nth < ne * NE) xs[q0 + u * nth] = v[u];
  }
  __syncthreads();
  using CT = const __attribute__((address_space(4))) T;
  CT* __restrict__ Ls = (CT*)L.Ls;
#pragma unroll 1
  for (int d = 0; d < DIM; ++d) {
    // line (el, o1, o2): o1, o2 the other directions' indices in increasing direction order
    const int st = d == 0 ? 1 : (d == 1 ? NP : NP * NP);
    constexpr int CH = PN ? NP : 1;  // work items per line
    for (int qq = tid; qq < ne * NLN * CH; qq += nth) {
      const int q = PN ? qq / NP : qq;
      const int el = q / NLN, ln = q - el * NLN;
      const int o1 = ln % NP, o2 = DIM == 3 ? ln / NP : 0;
      int base;
      T fac = two[el][d];
      if (d == 0) {
        base = (o2 * NP + o1) * NP;
        fac *= half[el][1] * srho[o1];
        if (DIM == 3) fac *= half[el][2] * srho[o2];
      } else if (d == 1) {
        base = o2 * NP * NP + o1;
        fac *= half[el][0] * srho[o1];
        if (DIM == 3) fac *= half[el][2] * srho[o2];
      } else {
        base = o2 * NP + o1;
        fac *= half[el][0] * srho[o1] * half[el][1] * srho[o2];
      }
      const T* src = xs + el * NE + base;
      T* dst = acc + el * NE + base;
      if constexpr (PN) {
        const int i = qq - q * NP;
        const T* lrow = SLS ? nullptr : sLs + i * NP;
        T s = T(0);
#pragma unroll
        for (int a = 0; a < NP; ++a) s += (SLS ? L.Ls[i * NP + a] : lrow[a]) * src[a * st];
        s *= fac;
        dst[i * st] = d == 0 ? s : dst[i * st] + s;
      } else {
        T v[NP];
#pragma unroll
        for (int a = 0; a < NP; ++a) v[a] = src[a * st];
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          T s = T(0);
#pragma unroll
          for (int a = 0; a < NP; ++a) s += (SLS ? (T)Ls[i * NP + a] : sLs[i * NP + a]) * v[a];
          s *= fac;
          dst[i * st] = d == 0 ? s : dst[i * st] + s;
        }
      }
    }
    __syncthreads();
  }
  for (int q = tid; q < ne * NE; q += nth) w[(int64_t)e0 * NE + q] = acc[q];
}

// y = A x (MODE 0) or y = f - A x (MODE 1) in one launch, each element
// computing the lattice nodes it owns (local index below P in every
// direction: every node has exactly one owner).  Per direction the assembled
// 1D row at an owned node is the element's own row of (2/dx) L^s, plus at its
// first node (shared with the left neighbour along that direction) row P of
// the neighbour's, applied to the neighbour's line read from global memory
// (L2); the other directions contribute the assembled lumped masses.  The
// element's closed tile is staged in LDS; then one thread per owned column
// along the last direction computes all DIM directional terms of the column's
// nodes (its own column with the rows of L^s as uniform operands, the other
// directions' lines from the tile with the thread's fixed rows in registers),
// so no partial sums go through LDS and the block needs only the tile.
template <int NP, int DIM>
constexpr int se_owned_bytes() {  // LDS per element
  return (ipow(NP, DIM) + DIM * ipow(NP - 1, DIM - 1)) * 8 + 3 * NP * 24 + 24;
}
template <int NP, int DIM>
constexpr int se_owned_epb() {  // a thread per owned column, 256 threads, within 64 KB of LDS
  return imax(1, imin(256 / ipow(NP - 1, DIM - 1), 64 * 1024 / se_owned_bytes<NP, DIM>()));
}
template <class T, int DIM, int NP>
__global__ void __launch_bounds__(256) se_owned_kernel(LevelDev<T> L, int mode, const T* __restrict__ x,
                                                       const T* __restrict__ f, T* __restrict__ y, int nblk,
                                                       int epb) {
  constexpr int P = NP - 1, NE = ipow(NP, DIM), NLN = ipow(P, DIM - 1);
  constexpr int EPB = se_owned_epb<NP, DIM>();
  static_assert(EPB * NLN <= 256, "one owned column per thread of a 256-thread block");
  __shared__ T xs[EPB * NE];
  __shared__ T lft[EPB][DIM][NLN];      // neighbour terms at the owned first nodes, per direction
  __shared__ int64_t off[EPB][3][NP];   // own closed tile
  __shared__ int64_t offl[EPB][3][NP];  // left neighbour's nodes along each direction (-1: none)
  __shared__ T mass[EPB][3][NP];        // assembled lumped mass at local index i < P
  __shared__ T two[EPB][3];
  __shared__ T sLs[NP * NP];
  const int blk = xcd_block(nblk);
  if (blk < 0 || inactive(L.active)) return;
  const int e0 = blk * epb, ne = imin(imin(epb, EPB), L.n_elem - e0);
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int q = tid; q < NP * NP; q += nth) sLs[q] = L.Ls[q];
  const int N1 = L.dir[0].N, N2 = L.dir[1].N;
  // element index along direction d of element e
  const auto mdir = [&](int e, int d) -> int {
    return d == 0 ? e % N1 : (d == 1 ? (DIM == 3 ? (e / N1) % N2 : e / N1) : e / (N1 * N2));
  };
  int64_t st[3];
  se_strides(L, st);
  // lattice offsets of the closed tile's nodes and of the left neighbour's
  // (integer work only, so the gather can start after one barrier)
  for (int q = tid; q < ne * 3 * NP; q += nth) {
    const int el = q / (3 * NP), rem = q - el * 3 * NP, d = rem / NP, i = rem - d * NP;
    if (d >= DIM) {
      off[el][d][i] = offl[el][d][i] = 0;
      continue;
    }
    const int md = mdir(e0 + el, d);
    const DirDev<T>& dd = L.dir[d];
    const bool hasl = dd.periodic || md > 0;
    const int ml = md == 0 ? dd.N - 1 : md - 1;
    const int s0 = se_stored(md * P + i, P, dd.N, dd.periodic);
    off[el][d][i] = s0 < 0 ? -1 : s0 * st[d];
    const int s1 = hasl ? se_stored(ml * P + i, P, dd.N, dd.periodic) : -1;
    offl[el][d][i] = s1 < 0 ? -1 : s1 * st[d];
  }
  // assembled lumped masses and 2/dx factors (global loads: issued behind the
  // gather's first group)
  const auto coef_tables = [&]() {
    for (int q = tid; q < ne * 3 * NP; q += nth) {
      const int el = q / (3 * NP), rem = q - el * 3 * NP, d = rem / NP, i = rem - d * NP;
      if (d >= DIM) {
        mass[el][d][i] = T(1);
        if (i == 0) two[el][d] = T(0);
        continue;
      }
      const int md = mdir(e0 + el, d);
      const DirDev<T>& dd = L.dir[d];
      const bool hasl = dd.periodic || md > 0;
      const int ml = md == 0 ? dd.N - 1 : md - 1;
      const T h = dd.ecoef[md * ECOEF_N + E_HALF_DX];
      T mv = h * L.rho[i];
      if (i == 0 && hasl) mv += dd.ecoef[ml * ECOEF_N + E_HALF_DX] * L.rho[P];
      mass[el][d][i] = mv;
      if (i == 0) two[el][d] = dd.ecoef[md * ECOEF_N + E_TWO_DX];
    }
  };
  __syncthreads();
  using CT = const __attribute__((address_space(4))) T;
  CT* __restrict__ Ls = (CT*)L.Ls;
  // neighbour term of direction d at owned face node (o1, o2) of the other
  // directions (increasing order): twol * (row P of L^s) . (the left
  // neighbour's line), 0 without a stored shared node (the neighbour's own
  // first node may be a dropped Dirichlet node, which reads as 0).  At most
  // DIM entries per thread.
  const auto neighbour_terms = [&]() {
#pragma unroll
    for (int r = 0; r < DIM; ++r) {
      const int q = tid + r * nth;
      if (q >= ne * DIM * NLN) break;
      const int el = q / (DIM * NLN), rem = q - el * DIM * NLN, d = rem / NLN, fi = rem - d * NLN;
      const int o1 = fi % P, o2 = DIM == 3 ? fi / P : 0;
      const int da = d == 0 ? 1 : 0, db = d == 2 ? 1 : 2;
      T left = T(0);
      const int64_t oa = off[el][da][o1], ob = DIM == 3 ? off[el][db][o2] : 0;
      if (offl[el][d][P] >= 0 && (oa | ob) >= 0) {  // a stored shared node: the neighbour exists
        const DirDev<T>& dd = L.dir[d];
        const int md = mdir(e0 + el, d), ml = md == 0 ? dd.N - 1 : md - 1;
        const T twol = dd.ecoef[ml * ECOEF_N + E_TWO_DX];
        const T* xl = x + oa + ob;
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          const int64_t oo = offl[el][d][a];
          T xv = T(0);
          if (oo >= 0) xv = xl[oo];
          left += (T)Ls[P * NP + a] * xv;
        }
        left *= twol;
      }
      lft[el][d][fi] = left;
    }
  };
  // the closed tiles, GU loads per thread in flight; the neighbour terms' loads
  // are issued behind the first group's, so both wait on one memory latency
  constexpr int GU = 12;
  for (int q0 = tid; q0 < ne * NE; q0 += GU * nth) {
    T v[GU];
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int q = q0 + u * nth;
      const int qq = q < ne * NE ? q : 0;
      const int el = qq / NE, loc = qq - el * NE;
      const int i = loc % NP, j = (loc / NP) % NP, k = DIM == 3 ? loc / (NP * NP) : 0;
      const int64_t a = off[el][0][i], b = off[el][1][j], c = off[el][2][k];
      const bool ok = q < ne * NE && (a | b | c) >= 0;
      T t = T(0);
      if (ok) t = x[a + b + c];
      v[u] = t;
    }
    if (q0 == tid) {
      neighbour_terms();
      coef_tables();
    }
#pragma unroll
    for (int u = 0; u < GU; ++u)
      if (q0 + u * nth < ne * NE) xs[q0 + u * nth] = v[u];
  }
  if (tid >= ne * NE) {  // threads without a tile entry
    neighbour_terms();
    coef_tables();
  }
  __syncthreads();
  // thread per owned column along direction DIM - 1: (i, j) in 3D, i in 2D
  for (int q = tid; q < ne * NLN; q += nth) {
    const int el = q / NLN, c = q - el * NLN;
    const T* __restrict__ xe = xs + el * NE;
    const int i = c % P, j = DIM == 3 ? c / P : 0;
    T col[NP], Li[NP], Lj[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      col[a] = DIM == 3 ? xe[i + NP * j + NP * NP * a] : xe[i + NP * a];
      Li[a] = sLs[i * NP + a];
      Lj[a] = DIM == 3 ? sLs[j * NP + a] : T(0);
    }
    const int64_t oi = off[el][0][i], oj = DIM == 3 ? off[el][1][j] : 0;
    const T mi = mass[el][0][i], mj = DIM == 3 ? mass[el][1][j] : T(1);
    const T t0 = two[el][0], t1 = two[el][1], tc = two[el][DIM - 1];
#pragma unroll 2
    for (int k = 0; k < P; ++k) {  // the column's nodes (its index in direction DIM - 1)
      // direction 0: row i along (., j, k)
      T s0 = T(0);
#pragma unroll
      for (int a = 0; a < NP; ++a) s0 += Li[a] * (DIM == 3 ? xe[a + NP * j + NP * NP * k] : xe[a + NP * k]);
      s0 *= t0;
      if (i == 0) s0 += lft[el][0][DIM == 3 ? j + P * k : k];
      s0 *= DIM == 3 ? mj * mass[el][2][k] : mass[el][1][k];
      T sum = s0;
      if constexpr (DIM == 3) {
        // direction 1: row j along (i, ., k)
        T s1 = T(0);
#pragma unroll
        for (int a = 0; a < NP; ++a) s1 += Lj[a] * xe[i + NP * a + NP * NP * k];
        s1 *= t1;
        if (j == 0) s1 += lft[el][1][i + P * k];
        s1 *= mi * mass[el][2][k];
        sum += s1;
      }
      // the column's own direction: row k (uniform) along the column
      T sc = T(0);
#pragma unroll
      for (int a = 0; a < NP; ++a) sc += (T)Ls[k * NP + a] * col[a];
      sc *= tc;
      if (k == 0) sc += lft[el][DIM - 1][c];
      sc *= DIM == 3 ? mi * mj : mi;
      sum += sc;
      const int64_t ok = off[el][DIM - 1][k];
      if ((oi | oj | ok) >= 0) {
        const int64_t g = oi + oj + ok;
        y[g] = mode == 1 ? f[g] - sum : sum;
      }
    }
  }
}

// Stored index per direction of lattice entry q (direction 0 fastest), in
// 32-bit arithmetic wherever the level's vector allows it: a 64-bit integer
// division costs several times as many instructions.
template <class T, int DIM>
__device__ __forceinline__ void se_split(const LevelDev<T>& L, int64_t q, int s[3]) {
  s[0] = s[1] = s[2] = 0;
  if (L.n_dof <= 0x7fffffff) {
    uint32_t rest = (uint32_t)q;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const uint32_t nl = (uint32_t)L.dir[d].nl;
      s[d] = (int)(rest % nl);
      rest /= nl;
    }
  } else {
    int64_t rest = q;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      s[d] = (int)(rest % L.dir[d].nl);
      rest /= L.dir[d].nl;
    }
  }
}

// Lattice node q of level L: per direction the (element, local node) pairs of
// the elements sharing it (two at an element boundary, else one).
template <class T, int DIM>
__device__ __forceinline__ void se_node_owners(const LevelDev<T>& L, int64_t q, int cnt[3], int em[3][2],
                                               int lo[3][2]) {
  const int P = L.P;
  int sd[3];
  se_split<T, DIM>(L, q, sd);
  for (int d = 0; d < 3; ++d) {
    cnt[d] = 1;
    em[d][0] = 0;
    lo[d][0] = 0;
    if (d >= DIM) continue;
    const DirDev<T>& dd = L.dir[d];
    const int s = sd[d];
    const int g = dd.periodic ? s : s + 1;
    const int m = g / P, i = g - m * P;
    if (i != 0) {
      em[d][0] = m;
      lo[d][0] = i;
    } else {  // shared by element m - 1 (its node P) and element m (its node 0)
      em[d][0] = m == 0 ? dd.N - 1 : m - 1;  // m = 0 only on a periodic direction
      lo[d][0] = P;
      em[d][1] = m;
      lo[d][1] = 0;
      cnt[d] = 2;
    }
  }
}

// y = sum of the element copies (MODE 0), y = f - sum (MODE 1).  All 2^DIM
// candidate slots are loaded at once (empty ones masked off) and added in the
// fixed order direction 3, 2, 1.
template <class T, int DIM, int NP>
__global__ void __launch_bounds__(256) se_dss_kernel(LevelDev<T> L, const T* __restrict__ w,
                                                     const T* __restrict__ f, T* __restrict__ y, int mode) {
  if (inactive(L.active)) return;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.n_dof) return;
  constexpr int NE = ipow(NP, DIM), CZ = DIM == 3 ? 2 : 1;
  int cnt[3], em[3][2], lo[3][2];
  se_node_owners<T, DIM>(L, q, cnt, em, lo);
  const int N1 = L.dir[0].N, N2 = L.dir[1].N;
  T v[CZ][2][2];
#pragma unroll
  for (int c = 0; c < CZ; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const bool ok = a < cnt[0] && b < cnt[1] && c < cnt[2];
        const int64_t e = em[0][ok ? a : 0] + (int64_t)N1 * (em[1][ok ? b : 0] + (int64_t)N2 * em[2][ok ? c : 0]);
        const int64_t idx = e * NE + (lo[2][ok ? c : 0] * NP + lo[1][ok ? b : 0]) * NP + lo[0][ok ? a : 0];
        T t = T(0);
        if (ok) t = w[idx];
        v[c][b][a] = t;
      }
  T s = T(0);
#pragma unroll
  for (int c = 0; c < CZ; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a)
        if (a < cnt[0] && b < cnt[1] && c < cnt[2]) s += v[c][b][a];
  y[q] = mode == 1 ? f[q] - s : s;
}

// u (+)= sum over the element-centred patches covering each lattice node of
// their weighted corrections (buf: one NA^DIM tile per patch, patch index
// m1 + N1 (m2 + N2 m3), tile position t1 + NA (t2 + NA t3), patch m's tile
// starting at lattice position m P - N_O).  MAXC: most patches covering a node
// per direction (2 when 2 N_O < P, else 3).  All candidate slots are loaded at
// once (empty ones masked off); sum order direction 3, 2, 1 candidates, each
// in increasing patch index.
template <class T, int DIM, int MAXC>
__global__ void __launch_bounds__(256) se_combine_kernel(LevelDev<T> L, int NA, const T* __restrict__ buf,
                                                         T* __restrict__ u, int assign) {
  if (inactive(L.active)) return;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.n_dof) return;
  constexpr int CZ = DIM == 3 ? MAXC : 1;
  const int P = L.P, NO = L.NO;
  int cnt[3], pm[3][MAXC], tp[3][MAXC];
  int sd[3];
  se_split<T, DIM>(L, q, sd);
  for (int d = 0; d < 3; ++d) {
    cnt[d] = 0;
#pragma unroll
    for (int k = 0; k < MAXC; ++k) pm[d][k] = tp[d][k] = 0;
    if (d >= DIM) {
      cnt[d] = 1;
      continue;
    }
    const DirDev<T>& dd = L.dir[d];
    const int s = sd[d];
    const int g = dd.periodic ? s : s + 1;
    const int m0 = g / P;
#pragma unroll
    for (int k = -2; k <= 1; ++k) {
      const int m = m0 + k;
      const int t = g - (m * P - NO);
      const bool in = t >= 0 && t < NA && cnt[d] < MAXC && (dd.periodic || (m >= 0 && m < dd.N));
      if (in) {
        // m lies within two elements of the lattice: wrap by additions
        int mw = m < 0 ? m + dd.N : m;
        mw = mw < 0 ? mw + dd.N : (mw >= dd.N ? mw - dd.N : mw);
        pm[d][cnt[d]] = mw >= dd.N ? mw - dd.N : mw;
        tp[d][cnt[d]] = t;
        ++cnt[d];
      }
    }
  }
  const int N1 = L.dir[0].N, N2 = L.dir[1].N;
  const int64_t TS = DIM == 3 ? (int64_t)NA * NA * NA : (int64_t)NA * NA;
  T v[CZ][MAXC][MAXC];
#pragma unroll
  for (int c = 0; c < CZ; ++c)
#pragma unroll
    for (int b = 0; b < MAXC; ++b)
#pragma unroll
      for (int a = 0; a < MAXC; ++a) {
        const bool ok = a < cnt[0] && b < cnt[1] && c < cnt[2];
        const int64_t pid = pm[0][a] + (int64_t)N1 * (pm[1][b] + (int64_t)N2 * pm[2][c]);
        T t = T(0);
        if (ok) t = buf[pid * TS + ((int64_t)tp[2][c] * NA + tp[1][b]) * NA + tp[0][a]];
        v[c][b][a] = t;
      }
  T s = T(0);
#pragma unroll
  for (int c = 0; c < CZ; ++c)
#pragma unroll
    for (int b = 0; b < MAXC; ++b)
#pragma unroll
      for (int a = 0; a < MAXC; ++a)
        if (a < cnt[0] && b < cnt[1] && c < cnt[2]) s += v[c][b][a];
  u[q] = assign ? s : u[q] + s;
}

// One contraction pass of the element transfers along direction D: src has
// NOUT points along directions < D and NIN along the others; dst maps
// direction D to NOUT points with M (row-major, MT = false: dst_i = sum_a
// M[i][a] src_a with M NOUT x NIN; MT = true: dst_i = sum_a M[a][i] src_a with
// M NIN x NOUT).
template <class T, int DIM, int NIN, int NOUT, int D, bool MT>
__device__ __forceinline__ void se_xpass(const T* __restrict__ M, const T* __restrict__ src, T* __restrict__ dst) {
  constexpr int n0 = D > 0 ? NOUT : NIN, n1 = DIM >= 2 ? (D > 1 ? NOUT : NIN) : 1;
  constexpr int m0 = D == 0 ? NOUT : n0;
  constexpr int m1 = D == 1 ? NOUT : n1;
  constexpr int m2 = DIM == 3 ? (D == 2 ? NOUT : NIN) : 1;
  constexpr int SK = D == 0 ? 1 : (D == 1 ? n0 : n0 * n1);
  for (int q = threadIdx.x; q < m0 * m1 * m2; q += blockDim.x) {
    const int i0 = q % m0, i1 = (q / m0) % m1, i2 = q / (m0 * m1);
    const int io = D == 0 ? i0 : (D == 1 ? i1 : i2);
    const int base = (D == 0 ? 0 : i0) + (D == 1 ? 0 : i1) * n0 + (D == 2 ? 0 : i2) * n0 * n1;
    T s = T(0);
#pragma unroll 4
    for (int a = 0; a < NIN; ++a) s += (MT ? M[a * NOUT + io] : M[io * NIN + a]) * src[base + a * SK];
    dst[q] = s;
  }
}

// u_f += I u_c on the fine nodes each element owns.  Lf: the fine level (J is
// NPF x NPC); Lc: the coarse level.
template <class T, int DIM, int NPF, int NPC>
__global__ void __launch_bounds__(256) se_prolong_kernel(LevelDev<T> Lf, LevelDev<T> Lc, const T* __restrict__ uc,
                                                         T* __restrict__ uf, int nblk) {
  constexpr int NEF = ipow(NPF, DIM), NEC = ipow(NPC, DIM);
  __shared__ T ta[NEF], tb[NEF];
  __shared__ T sJ[NPF * NPC];
  __shared__ int64_t offc[1][3][NPC];
  __shared__ int64_t offf[1][3][NPF];
  const int e = xcd_block(nblk);
  if (e < 0 || inactive(Lf.active)) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int q = tid; q < NPF * NPC; q += nth) sJ[q] = Lf.J[q];
  se_elem_offsets<T, DIM, NPC, 1>(Lc, e, 1, offc);
  se_elem_offsets<T, DIM, NPF, 1>(Lf, e, 1, offf);
  __syncthreads();
  for (int q = tid; q < NEC; q += nth) {
    const int i = q % NPC, j = (q / NPC) % NPC, k = DIM == 3 ? q / (NPC * NPC) : 0;
    const int64_t a = offc[0][0][i], b = offc[0][1][j], c = offc[0][2][k];
    const bool ok = (a | b | c) >= 0;
    const T v = uc[ok ? a + b + c : 0];
    ta[q] = ok ? v : T(0);
  }
  __syncthreads();
  se_xpass<T, DIM, NPC, NPF, 0, false>(sJ, ta, tb);
  __syncthreads();
  se_xpass<T, DIM, NPC, NPF, 1, false>(sJ, tb, ta);
  __syncthreads();
  const T* res = ta;
  if constexpr (DIM == 3) {
    se_xpass<T, DIM, NPC, NPF, 2, false>(sJ, ta, tb);
    __syncthreads();
    res = tb;
  }
  constexpr int PF = NPF - 1;
  for (int q = tid; q < NEF; q += nth) {
    const int i = q % NPF, j = (q / NPF) % NPF, k = DIM == 3 ? q / (NPF * NPF) : 0;
    if (i == PF || j == PF || (DIM == 3 && k == PF)) continue;  // owned by the next element
    const int64_t a = offf[0][0][i], b = offf[0][1][j], c = offf[0][2][k];
    if ((a | b | c) < 0) continue;
    uf[a + b + c] += res[q];
  }
}

// wc_e = (J^T (x) J^T (x) J^T) (W r_f,e) per element (element-major coarse
// output): W halves a fine node per direction in which it lies on an element
// boundary (shared by two elements; dropped Dirichlet nodes read 0).
template <class T, int DIM, int NPF, int NPC>
__global__ void __launch_bounds__(256) se_restrict_kernel(LevelDev<T> Lf, const T* __restrict__ rf,
                                                          T* __restrict__ wc, int nblk) {
  constexpr int NEF = ipow(NPF, DIM), NEC = ipow(NPC, DIM);
  __shared__ T ta[NEF], tb[NEF];
  __shared__ T sJ[NPF * NPC];
  __shared__ int64_t offf[1][3][NPF];
  const int e = xcd_block(nblk);
  if (e < 0 || inactive(Lf.active)) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int q = tid; q < NPF * NPC; q += nth) sJ[q] = Lf.J[q];
  se_elem_offsets<T, DIM, NPF, 1>(Lf, e, 1, offf);
  __syncthreads();
  constexpr int PF = NPF - 1;
  for (int q = tid; q < NEF; q += nth) {
    const int i = q % NPF, j = (q / NPF) % NPF, k = DIM == 3 ? q / (NPF * NPF) : 0;
    const int64_t a = offf[0][0][i], b = offf[0][1][j], c = offf[0][2][k];
    const bool ok = (a | b | c) >= 0;
    T v = rf[ok ? a + b + c : 0];
    T wgt = T(1);
    if (i == 0 || i == PF) wgt *= T(0.5);
    if (j == 0 || j == PF) wgt *= T(0.5);
    if (DIM == 3 && (k == 0 || k == PF)) wgt *= T(0.5);
    ta[q] = ok ? wgt * v : T(0);
  }
  __syncthreads();
  se_xpass<T, DIM, NPF, NPC, 0, true>(sJ, ta, tb);
  __syncthreads();
  se_xpass<T, DIM, NPF, NPC, 1, true>(sJ, tb, ta);
  __syncthreads();
  const T* res = ta;
  if constexpr (DIM == 3) {
    se_xpass<T, DIM, NPF, NPC, 2, true>(sJ, ta, tb);
    __syncthreads();
    res = tb;
  }
  for (int q = tid; q < NEC; q += nth) wc[(int64_t)e * NEC + q] = res[q];
}

inline unsigned se_node_blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

// ------------------------------------------------------------------ launchers
template <class T, int DIM, int NP>
int se_apply_launch(const LevelDev<T>& L, int mode, const T* x, const T* f, T* y, T* ebuf, hipStream_t s) {
  if constexpr (DIM == 3 && NP > 17) {
    return -4;  // element tiles beyond LDS
  } else {
    if (mode != 0 && mode != 1) return -4;
    // owner-computes form (one launch, no element copies) on levels with many
    // lines; small levels keep the two-launch form, whose thread-per-output
    // variant has more parallel work
    if (NP >= 3 && (int64_t)L.n_elem * ipow(NP - 1, DIM - 1) >= 64 * 1024) {
      constexpr int EPBO = se_owned_epb<NP, DIM>();
      const int epb = imax(1, imin(EPBO, L.n_elem / 512));
      const int nb = (L.n_elem + epb - 1) / epb;
      hipLaunchKernelGGL((se_owned_kernel<T, DIM, NP>), dim3(xcd_grid(nb)), dim3(256), 0, s, L, mode, x, f, y, nb,
                         epb);
      return 0;
    }
    // elements per block: up to se_epb, fewer on small levels so that the
    // launch still has about 512 blocks
    constexpr int EPB = se_epb<NP, DIM>(), NLN = ipow(NP, DIM - 1);
    const int epb = imax(1, imin(EPB, L.n_elem / 512));
    const int nb = (L.n_elem + epb - 1) / epb;
    if ((int64_t)nb * epb * NLN < 128 * 1024) {  // fewer than ~128k lines: a thread per line and output
      const int th = imin(1024, round64(epb * NLN * NP));
      hipLaunchKernelGGL((se_elem_kernel<T, DIM, NP, true>), dim3(xcd_grid(nb)), dim3(th), 0, s, L, x, ebuf, nb, epb);
    } else {
      const int th = imin(1024, round64(epb * NLN));
      hipLaunchKernelGGL((se_elem_kernel<T, DIM, NP, false>), dim3(xcd_grid(nb)), dim3(th), 0, s, L, x, ebuf, nb,
                         epb);
    }
    hipLaunchKernelGGL((se_dss_kernel<T, DIM, NP>), dim3(se_node_blocks(L.n_dof)), dim3(256), 0, s, L,
                       (const T*)ebuf, f, y, mode);
    return 0;
  }
}

template <class T, int DIM>
int se_combine_launch(const LevelDev<T>& L, int NA, const T* buf, T* u, bool assign, hipStream_t s) {
  if (2 * L.NO < L.P)
    hipLaunchKernelGGL((se_combine_kernel<T, DIM, 2>), dim3(se_node_blocks(L.n_dof)), dim3(256), 0, s, L, NA, buf, u,
                       assign ? 1 : 0);
  else
    hipLaunchKernelGGL((se_combine_kernel<T, DIM, 3>), dim3(se_node_blocks(L.n_dof)), dim3(256), 0, s, L, NA, buf, u,
                       assign ? 1 : 0);
  return 0;
}

template <class T, int DIM, int NPF, int NPC>
int se_transfer_launch(const LevelDev<T>& Lf, const LevelDev<T>& Lc, bool restrict_, const T* in, T* out, T* ebuf,
                       hipStream_t s) {
  if constexpr (DIM == 3 && NPF > 17) {
    return -4;
  } else {
    const int nb = Lf.n_elem;
    if (restrict_) {
      hipLaunchKernelGGL((se_restrict_kernel<T, DIM, NPF, NPC>), dim3(xcd_grid(nb)), dim3(256), 0, s, Lf, in, ebuf,
                         nb);
      hipLaunchKernelGGL((se_dss_kernel<T, DIM, NPC>), dim3(se_node_blocks(Lc.n_dof)), dim3(256), 0, s, Lc,
                         (const T*)ebuf, (const T*)nullptr, out, 0);
    } else {
      hipLaunchKernelGGL((se_prolong_kernel<T, DIM, NPF, NPC>), dim3(xcd_grid(nb)), dim3(256), 0, s, Lf, Lc, in,
                         out, nb);
    }
    return 0;
  }
}

}  // namespace dgmg

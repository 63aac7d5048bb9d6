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
// One launch per direction D (in order 0, 1, 2), one thread per line of that
// direction, apply_lb<T>() lines per block: enough blocks to fill the chip
// although there are few elements.  Launch D adds the direction-D terms to y
// (launch 0 writes them); the last launch applies the mode: y = A x (MODE 0),
// y = f - A x accumulated as ((f - c0) - c1) - c2 so that y may alias f
// (MODE 1), y = A x with per-block partial sums of x.y (MODE 2).  The kernel
// boundaries order the three contributions: results are deterministic.
// Lines of direction 0 are contiguous in memory, so for D = 0 the block's
// lines of the element and of both neighbours are staged through LDS with
// coalesced loads (and the results stored the same way); lines of directions
// 1 and 2 are read directly (consecutive lanes, consecutive addresses).
// y must not alias x.
template <class T>
constexpr int apply_lb() {
  return sizeof(T) == 8 ? 64 : 128;
}

// Face data of every direction-0 line (element-major, line-major): its two end
// values and the two end derivatives, {v_0, v_P, D0 . v, DP . v}.  The
// block's lines are staged through LDS with coalesced loads.
template <class T, int NP>
__global__ void __launch_bounds__(128) apply_big_face0(LevelDev<T> L, const T* __restrict__ x,
                                                       T* __restrict__ face, int nblk) {
  constexpr int NE = NP * NP * NP, NLN = NP * NP, P = NP - 1, LB = apply_lb<T>();
  constexpr int CH = (NLN + LB - 1) / LB;
  __shared__ T sx[LB * NP], sD0[NP], sDP[NP];
  const int b = xcd_block(nblk);
  if (b < 0 || inactive(L.active)) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int q = tid; q < NP; q += nth) {
    sD0[q] = L.D[q];
    sDP[q] = L.D[P * NP + q];
  }
  const int e = b / CH, c0 = (b - e * CH) * LB, t = c0 + tid;
  const int nlines = imin(LB, NLN - c0);
  const int64_t o = (int64_t)e * NE + (int64_t)c0 * NP;
  staged_copy<T, LB, LB * NP>([&](int q) { return x[o + q]; }, [&](int q, T v) { sx[q] = v; }, nlines * NP);
  __syncthreads();
  if (t < NLN) {
    T d0 = 0, dP = 0;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const T v = sx[tid * NP + k];
      d0 += sD0[k] * v;
      dP += sDP[k] * v;
    }
    T* fo = face + ((int64_t)e * NLN + t) * 4;
    fo[0] = sx[tid * NP];
    fo[1] = sx[tid * NP + P];
    fo[2] = d0;
    fo[3] = dP;
  }
}

// face: direction-0 face data of every element (apply_big_face0), D = 0 only.
template <class T, int NP, int MODE, int D>
__global__ void __launch_bounds__(128) apply_big_kernel(LevelDev<T> L, const T* __restrict__ x, const T* f, T* y,
                                                        const T* __restrict__ face, double* __restrict__ part,
                                                        int nblk) {
  constexpr int NE = NP * NP * NP, NLN = NP * NP, P = NP - 1, LB = apply_lb<T>();
  constexpr int CH = (NLN + LB - 1) / LB;  // line chunks per element
  constexpr int SX = D == 0 ? LB * NP : 1;
  __shared__ double red[16];
  __shared__ T srho[NP];
  __shared__ T sx[SX];
  const int b = xcd_block(nblk);
  if (b < 0 || inactive(L.active)) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int q = tid; q < NP; q += nth) srho[q] = L.rho[q];
  // the stiffness matrix and end-derivative rows: uniform addresses in the
  // constant address space, read with scalar loads into SGPR operands
  using CT = const __attribute__((address_space(4))) T;
  CT* __restrict__ sLs = (CT*)L.Ls;
  CT* __restrict__ sD0 = (CT*)L.D;
  CT* __restrict__ sDP = (CT*)(L.D + P * NP);
  const int e = b / CH, c0 = (b - e * CH) * LB, t = c0 + tid;
  const int nlines = imin(LB, NLN - c0);
  const int N1 = L.dir[0].N, N2 = L.dir[1].N;
  int m[3];
  m[0] = e % N1;
  m[1] = (e / N1) % N2;
  m[2] = e / (N1 * N2);
  const int64_t g0 = (int64_t)e * NE;
  const DirDev<T> dd = L.dir[D];
  const int estride = D == 0 ? 1 : (D == 1 ? N1 : N1 * N2);
  const int nl = dd.nbr[2 * m[D]], nr = dd.nbr[2 * m[D] + 1];
  const int el = e + (nl >= 0 ? nl - m[D] : 0) * estride, er = e + (nr >= 0 ? nr - m[D] : 0) * estride;
  if constexpr (D == 0) {  // the block's lines are NP * nlines consecutive values
    const int64_t o = g0 + (int64_t)c0 * NP;
    staged_copy<T, LB, SX>([&](int q) { return x[o + q]; }, [&](int q, T v) { sx[q] = v; }, nlines * NP);
  }
  __syncthreads();
  double acc = 0.0;
  if (t < NLN) {
    const T* c = dd.ecoef + m[D] * ECOEF_N;
    const int da = D == 0 ? 1 : 0, db = D == 2 ? 1 : 2;
    const T ha = L.dir[da].ecoef[m[da] * ECOEF_N + E_HALF_DX], hb = L.dir[db].ecoef[m[db] * ECOEF_N + E_HALF_DX];
    const int ia = t % NP, ib = t / NP;
    const int base = D == 0 ? t * NP : (D == 1 ? ia + ib * NP * NP : t);
    const int stride = D == 0 ? 1 : (D == 1 ? NP : NP * NP);
    T v[NP];
    T d0 = 0, dP = 0, dL = 0, dR = 0, wlP = 0, wr0 = 0;
    if constexpr (D == 0) {
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        v[k] = sx[tid * NP + k];
        d0 += sD0[k] * v[k];
        dP += sDP[k] * v[k];
      }
      const T* fl_ = face + ((int64_t)el * NLN + t) * 4;  // left neighbour: its value and derivative at i = P
      const T* fr_ = face + ((int64_t)er * NLN + t) * 4;  // right neighbour: at i = 0
      wlP = fl_[1];
      dL = fl_[3];
      wr0 = fr_[0];
      dR = fr_[2];
    } else {
      const int64_t gl = (int64_t)el * NE, gr = (int64_t)er * NE;
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        v[k] = x[g0 + base + k * stride];
        const T wlk = x[gl + base + k * stride], wrk = x[gr + base + k * stride];
        if (k == P) wlP = wlk;
        if (k == 0) wr0 = wrk;
        d0 += sD0[k] * v[k];
        dP += sDP[k] * v[k];
        dL += sDP[k] * wlk;
        dR += sD0[k] * wrk;
      }
    }
    const T ml = nl >= 0 ? T(1) : T(0), mr = nr >= 0 ? T(1) : T(0);
    const T uL = ml * wlP, uR = mr * wr0;
    dL *= ml;
    dR *= mr;
    const T jl = v[0] - uL, jr = v[P] - uR;
    const T fl = c[E_CL] * d0 + c[E_CNL] * dL + c[E_BL] * jl;
    const T fr = -c[E_CR] * dP - c[E_CNR] * dR + c[E_BR] * jr;
    const T cl = c[E_CL] * jl, cr = c[E_CR] * jr, tdx = c[E_TWO_DX];
    const T mo = ha * srho[ia] * hb * srho[ib];
#pragma unroll 1
    for (int i = 0; i < NP; ++i) {
      const int iu = __builtin_amdgcn_readfirstlane(i);
      T s = 0;
#pragma unroll
      for (int k = 0; k < NP; ++k) s += sLs[iu * NP + k] * v[k];
      T o = tdx * s + cl * sD0[iu] - cr * sDP[iu];
      if (i == 0) o += fl;
      if (i == P) o += fr;
      const T val = mo * o;
      if constexpr (D == 0) {
        sx[tid * NP + i] = val;  // this thread's own line: stored below, coalesced
      } else {
        const int64_t idx = g0 + base + i * stride;
        if (MODE == 1) {
          y[idx] = y[idx] - val;
        } else {
          const T tot = y[idx] + val;
          y[idx] = tot;
          // v_i read again from x: indexing v by the rolled loop counter
          // would put the line in scratch memory
          if (MODE == 2 && D == 2) acc += (double)x[g0 + base + i * stride] * (double)tot;
        }
      }
    }
  }
  if constexpr (D == 0) {
    __syncthreads();
    const int64_t o = g0 + (int64_t)c0 * NP;
    if constexpr (MODE == 1)
      staged_copy<T, LB, SX>([&](int q) { return f[o + q]; }, [&](int q, T v) { y[o + q] = v - sx[q]; }, nlines * NP);
    else
      for (int q = tid; q < nlines * NP; q += nth) y[o + q] = sx[q];
  }
  if constexpr (MODE == 2 && D == 2) {
    const double sum = block_sum(acc, red);
    if (tid == 0) part[b] = sum;
  }
}

// Partial sums written by the MODE-2 apply of a large-element level.
template <class T, int NP>
constexpr int apply_big_blocks_per_elem() {
  return (NP * NP + apply_lb<T>() - 1) / apply_lb<T>();
}

template <class T, int NP, int MODE>
void apply_big_dirs(const LevelDev<T>& L, const T* x, const T* f, T* y, T* face, double* part, int nblk,
                    hipStream_t s) {
  dim3 grid(xcd_grid(nblk)), block(apply_lb<T>());
  hipLaunchKernelGGL((apply_big_face0<T, NP>), grid, block, 0, s, L, x, face, nblk);
  hipLaunchKernelGGL((apply_big_kernel<T, NP, MODE, 0>), grid, block, 0, s, L, x, f, y, face, part, nblk);
  hipLaunchKernelGGL((apply_big_kernel<T, NP, MODE, 1>), grid, block, 0, s, L, x, f, y, face, part, nblk);
  hipLaunchKernelGGL((apply_big_kernel<T, NP, MODE, 2>), grid, block, 0, s, L, x, f, y, face, part, nblk);
}

// Scratch elements of the large-element apply (direction-0 face data).
inline int64_t apply_big_scratch(int n_elem, int NP) { return (int64_t)4 * n_elem * NP * NP; }

template <class T, int NP>
int apply_big_launch(const LevelDev<T>& L, int mode, const T* x, const T* f, T* y, T* scratch, double* part,
                     int* nblk_out, hipStream_t s) {
  const int nblk = L.n_elem * apply_big_blocks_per_elem<T, NP>();
  if (nblk_out) *nblk_out = nblk;
  if (mode == 0)
    apply_big_dirs<T, NP, 0>(L, x, f, y, scratch, part, nblk, s);
  else if (mode == 1)
    apply_big_dirs<T, NP, 1>(L, x, f, y, scratch, part, nblk, s);
  else
    apply_big_dirs<T, NP, 2>(L, x, f, y, scratch, part, nblk, s);
  return 0;
}

// ================================================================ p-transfers
// Restriction out_c = (J^T x J^T x J^T) in_f in two kernels: the slowest
// direction through the scratch tmp [e][k'][j][i], then the two fast
// directions per (element, k') plane in LDS.  Prolongation out_f += (J x J x J)
// in_c: the two fast directions per coarse plane into tmp [e][k][j][i], then
// the slowest direction accumulated into out.
// One thread per (element, fine column ji): the column's NPF values are read
// once and give all NPC outputs; the rows of J are uniform, read by scalar
// loads (each output still sums k = 0, 1, ... in order).
template <class T, int NPF, int NPC>
__global__ void __launch_bounds__(256) restrict_z_kernel(const T* __restrict__ J, int n_elem,
                                                         const T* __restrict__ in, T* __restrict__ tmp,
                                                         const int* __restrict__ active) {
  if (inactive(active)) return;
  constexpr int PL = NPF * NPF, NEF = NPF * PL, PER = NPC * PL;
  using CT = const __attribute__((address_space(4))) T;
  CT* __restrict__ Jc = (CT*)J;
  const int64_t total = (int64_t)n_elem * PL;
  // one column per thread (no grid-stride loop: J's rows would be hoisted out of it)
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < total) {
    const int64_t e = q / PL;
    const int ji = (int)(q - e * PL);
    const T* src = in + e * NEF + ji;
    T v[NPF];
#pragma unroll
    for (int k = 0; k < NPF; ++k) v[k] = src[k * PL];
    T acc[NPC];
#pragma unroll
    for (int kc = 0; kc < NPC; ++kc) acc[kc] = T(0);
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
#pragma unroll
      for (int kc = 0; kc < NPC; ++kc) acc[kc] += Jc[k * NPC + kc] * v[k];
      // two rows of J in scalar registers at a time (no hoisting of all of J)
      if (k % 2 == 1) __builtin_amdgcn_sched_barrier(0);
    }
    T* dst = tmp + e * PER + ji;
#pragma unroll
    for (int kc = 0; kc < NPC; ++kc) dst[kc * PL] = acc[kc];
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
  staged_copy<T, 256, PL>([&](int q) { return src[q]; }, [&](int q, T v) { pl[q] = v; });
  staged_copy<T, 256, NPF * NPC>([&](int q) { return J[q]; }, [&](int q, T v) { sJ[q] = v; });
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
  staged_copy<T, 256, NPC * NPC>([&](int q) { return src[q]; }, [&](int q, T v) { pl[q] = v; });
  staged_copy<T, 256, NPF * NPC>([&](int q) { return J[q]; }, [&](int q, T v) { sJ[q] = v; });
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

// One thread per (element, column ji): the NPC coarse values of the column are
// read once and update all NPF fine values (each sums kc = 0, 1, ... in order).
template <class T, int NPF, int NPC>
__global__ void __launch_bounds__(256) prolong_z_kernel(const T* __restrict__ J, int n_elem,
                                                        const T* __restrict__ tmp, T* __restrict__ out,
                                                        const int* __restrict__ active) {
  if (inactive(active)) return;
  constexpr int PL = NPF * NPF, NEF = NPF * PL, TPE = NPC * PL;
  using CT = const __attribute__((address_space(4))) T;
  CT* __restrict__ Jc = (CT*)J;
  const int64_t total = (int64_t)n_elem * PL;
  // one column per thread (no grid-stride loop: J's rows would be hoisted out of it)
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < total) {
    const int64_t e = q / PL;
    const int ji = (int)(q - e * PL);
    const T* src = tmp + e * TPE + ji;
    T w[NPC];
#pragma unroll
    for (int kc = 0; kc < NPC; ++kc) w[kc] = src[kc * PL];
    T* dst = out + e * NEF + ji;
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
      T s = 0;
#pragma unroll
      for (int kc = 0; kc < NPC; ++kc) s += Jc[k * NPC + kc] * w[kc];
      dst[k * PL] += s;
      // two rows of J in scalar registers at a time (no hoisting of all of J)
      if (k % 2 == 1) __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Scratch elements the two-kernel transfer needs (n_elem NPC NPF^2).
inline int64_t transfer_big_scratch(int n_elem, int NPF, int NPC) { return (int64_t)n_elem * NPC * NPF * NPF; }

template <class T, int NPF, int NPC>
int transfer_big_launch(const T* J, int n_elem, bool restrict_, const T* in, T* out, T* tmp, const int* active,
                        hipStream_t s) {
  // z stages: one thread per (element, column)
  const int64_t ncol = (int64_t)n_elem * NPF * NPF;  // < 2^31 / NPF columns
  const unsigned gz = (unsigned)((ncol + 255) / 256);
  const unsigned gp = (unsigned)(n_elem * NPC);
  if (restrict_) {
    hipLaunchKernelGGL((restrict_z_kernel<T, NPF, NPC>), dim3(gz), dim3(256), 0, s, J, n_elem, in, tmp, active);
    hipLaunchKernelGGL((restrict_xy_kernel<T, NPF, NPC>), dim3(gp), dim3(256), 0, s, J, n_elem, tmp, out, active);
  } else {
    hipLaunchKernelGGL((prolong_xy_kernel<T, NPF, NPC>), dim3(gp), dim3(256), 0, s, J, n_elem, in, tmp, active);
    hipLaunchKernelGGL((prolong_z_kernel<T, NPF, NPC>), dim3(gz), dim3(256), 0, s, J, n_elem, tmp, out, active);
  }
  return 0;
}

// ================================================================ FDM patch solve
// In-place line contraction on a 2D LDS array: for each of `lines` lines v
// (element k at tile[line * ls + k * ks]) out_j = sum_k B[k][j] v_k, B row-major
// LEN x LEN in global memory, on 16x16x4 matrix-core products (see Mfma).
// Column split for the long lines of large tiles (lines <= 64,
// LEN <= 64, at least (LEN + 15) / 16 waves): wave w computes output columns
// j in [16 w, 16 w + 16) for every line block, holding only its 16 x LEN slice
// of B (LEN / 4 values per lane) and all results in registers; after a
// barrier the waves write their columns back in place.  Every wave, active or
// not, reaches the barrier.
template <class T, int LEN>
__device__ __forceinline__ void mfma_lines_cols(T* __restrict__ tile, int lines, int ls, int ks_,
                                                const T* __restrict__ Bm) {
  constexpr int KS = (LEN + 3) / 4, NB = (LEN + 15) / 16, MBX = 4;
  using M = Mfma<T>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int MB = (lines + 15) / 16;
  const int nb = wave;
  const bool act = nb < NB;  // wave-uniform
  typename M::acc_t acc[MBX];
#pragma unroll
  for (int mb = 0; mb < MBX; ++mb) acc[mb] = typename M::acc_t{0, 0, 0, 0};
  if (act) {
    T b[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + lk, j = nb * 16 + li;
      b[ks] = (k < LEN && j < LEN) ? Bm[k * LEN + j] : T(0);
    }
#pragma unroll
    for (int mb = 0; mb < MBX; ++mb) {
      if (mb < MB) {
        const int line = mb * 16 + li;
        const bool lv = line < lines;
        const int base = lv ? line * ls : 0;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const int k = 4 * ks + lk;
          const T a = (lv && k < LEN) ? tile[base + k * ks_] : T(0);
          acc[mb] = M::op(b[ks], a, acc[mb]);
        }
      }
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int mb = 0; mb < MBX; ++mb) {
      const int line = mb * 16 + li;
      if (mb < MB && line < lines) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = nb * 16 + M::row(lk, r);
          if (j < LEN) tile[line * ls + j * ks_] = acc[mb][r];
        }
      }
    }
  }
}

// Per-patch data of the three stages; ND = the sweep normal (-1: element-
// centred), all tile lengths compile-time: len[d] = NA for d = ND, else NL.
template <class T, int NA, int NL, int ND>
struct BigPatch {
  static constexpr int L0 = ND == 0 ? NA : NL, L1 = ND == 1 ? NA : NL, L2 = ND == 2 ? NA : NL;
  static constexpr int TS = L0 * L1 * L2;
  int p[3];
  const int* go[3];  // gather offsets of the patch positions (-1 outside)
  const T* w[3];
  const T* lam[3];
  const T* S[3];
  const T* ST[3];
  __device__ __forceinline__ BigPatch(const LevelDev<T>& L, int pid, int npx, int npy) {
    p[0] = pid % npx;
    p[1] = (pid / npx) % npy;
    p[2] = pid / (npx * npy);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const DirDev<T>& dd = L.dir[d];
      const bool fc = d == ND;
      go[d] = fc ? dd.goff_fc + p[d] * NA : dd.goff_ec + p[d] * NL;
      w[d] = fc ? dd.w_fc + p[d] * NA : dd.w_ec + p[d] * NL;
      lam[d] = fc ? dd.lam_fc + p[d] * NA : dd.lam_ec + p[d] * NL;
      S[d] = fc ? dd.S_fc + (int64_t)p[d] * NA * NA : dd.S_ec + (int64_t)p[d] * NL * NL;
      ST[d] = fc ? dd.ST_fc + (int64_t)p[d] * NA * NA : dd.ST_ec + (int64_t)p[d] * NL * NL;
    }
  }
};

constexpr int big_pitch(int n) { return n % 2 == 0 ? n + 1 : n; }

// Threads of the stage launches (compile-time: the copies below unroll over them).
constexpr int BIG_AC_THREADS = 256;
template <int L2>
constexpr int big_b_threads() {
  return 64 * ((L2 + 15) / 16);  // one wave per output column block of direction 2
}

// Stage A: block per (patch, o2).  Gather the plane o2 of R_s r, forward
// transform along directions 0 and 1, store it in the patch's slot
// (grid-natural order (o2 L1 + o1) L0 + o0).
template <class T, int NA, int NL, int ND>
__global__ void __launch_bounds__(256) fdm_big_a(LevelDev<T> L, const T* __restrict__ r, T* __restrict__ out,
                                                 int npx, int npy, int npz) {
  using Q = BigPatch<T, NA, NL, ND>;
  constexpr int N0 = Q::L0, N1 = Q::L1, N2 = Q::L2, PT = big_pitch(N0);
  __shared__ T pl[N1 * PT];
  __shared__ int g0[N0], g1[N1];
  const int npatch = npx * npy * npz;
  const int bid = xcd_block(npatch * N2);
  if (bid < 0 || inactive(L.active)) return;
  const int pid = bid / N2, o2 = bid - pid * N2;
  const Q q(L, pid, npx, npy);
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int o = tid; o < N0; o += nth) g0[o] = q.go[0][o];
  for (int o = tid; o < N1; o += nth) g1[o] = q.go[1][o];
  const int gz = q.go[2][o2];
  __syncthreads();
  // positions outside a Dirichlet domain read r[0] and store 0
  const auto gidx = [&](int e) {
    const int o1 = e / N0, o0 = e - o1 * N0;
    const int a = g0[o0], b = g1[o1];
    return (gz | a | b) >= 0 ? gz + a + b : -1;
  };
  staged_copy<T, BIG_AC_THREADS, N0 * N1>([&](int e) { const int i = gidx(e); return r[i >= 0 ? i : 0]; },
                                       [&](int e, T v) {
                                         const int o1 = e / N0, o0 = e - o1 * N0;
                                         pl[o1 * PT + o0] = gidx(e) >= 0 ? v : T(0);
                                       });
  __syncthreads();
  mfma_lines_cols<T, N0>(pl, N1, PT, 1, q.S[0]);  // rows: direction 0
  __syncthreads();
  mfma_lines_cols<T, N1>(pl, N0, 1, PT, q.S[1]);  // columns: direction 1
  __syncthreads();
  T* dst = out + (int64_t)pid * Q::TS + (int64_t)o2 * N0 * N1;
  staged_copy<T, BIG_AC_THREADS, N0 * N1>([&](int e) { const int o1 = e / N0; return pl[o1 * PT + e - o1 * N0]; },
                                       [&](int e, T v) { dst[e] = v; });
}

// Stage B: block per (patch, o1).  Along direction 2: forward transform, scale
// by 1 / (lam0 + lam1 + lam2), backward transform; in place in the slot.
template <class T, int NA, int NL, int ND>
__global__ void __launch_bounds__(256) fdm_big_b(LevelDev<T> L, T* __restrict__ out, int npx, int npy, int npz) {
  using Q = BigPatch<T, NA, NL, ND>;
  constexpr int N0 = Q::L0, N1 = Q::L1, N2 = Q::L2, PT = big_pitch(N0);
  __shared__ T pl[N2 * PT];
  __shared__ T l0[N0], l2[N2];
  const int npatch = npx * npy * npz;
  const int bid = xcd_block(npatch * N1);
  if (bid < 0 || inactive(L.active)) return;
  const int pid = bid / N1, o1 = bid - pid * N1;
  const Q q(L, pid, npx, npy);
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int o = tid; o < N0; o += nth) l0[o] = q.lam[0][o];
  for (int o = tid; o < N2; o += nth) l2[o] = q.lam[2][o];
  const T l1 = q.lam[1][o1];
  T* slot = out + (int64_t)pid * Q::TS + (int64_t)o1 * N0;
  constexpr int64_t ZST = (int64_t)N0 * N1;
  constexpr int NTB = big_b_threads<N2>();
  staged_copy<T, NTB, N0 * N2>([&](int e) { const int o2 = e / N0; return slot[o2 * ZST + e - o2 * N0]; },
                            [&](int e, T v) { const int o2 = e / N0; pl[o2 * PT + e - o2 * N0] = v; });
  __syncthreads();
  mfma_lines_cols<T, N2>(pl, N0, 1, PT, q.S[2]);
  __syncthreads();
  for (int e = tid; e < N0 * N2; e += nth) {
    const int o2 = e / N0, o0 = e - o2 * N0;
    const int i = o2 * PT + o0;
    const T den = l0[o0] + l1 + l2[o2];
    if constexpr (DGMG_FDM_DIV_NR) pl[i] = div_nr(pl[i], den);  // Newton-refined reciprocal
    else pl[i] = pl[i] / den;
  }
  __syncthreads();
  mfma_lines_cols<T, N2>(pl, N0, 1, PT, q.ST[2]);
  __syncthreads();
  staged_copy<T, NTB, N0 * N2>([&](int e) { const int o2 = e / N0; return pl[o2 * PT + e - o2 * N0]; },
                            [&](int e, T v) { const int o2 = e / N0; slot[o2 * ZST + e - o2 * N0] = v; });
}

// Stage C: block per (patch, o2).  Backward transform along directions 1 and 0,
// multiply by the weights w0 w1 w2; in place in the slot.
template <class T, int NA, int NL, int ND>
__global__ void __launch_bounds__(256) fdm_big_c(LevelDev<T> L, T* __restrict__ out, int npx, int npy, int npz) {
  using Q = BigPatch<T, NA, NL, ND>;
  constexpr int N0 = Q::L0, N1 = Q::L1, N2 = Q::L2, PT = big_pitch(N0);
  __shared__ T pl[N1 * PT];
  __shared__ T w0[N0], w1[N1];
  const int npatch = npx * npy * npz;
  const int bid = xcd_block(npatch * N2);
  if (bid < 0 || inactive(L.active)) return;
  const int pid = bid / N2, o2 = bid - pid * N2;
  const Q q(L, pid, npx, npy);
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int o = tid; o < N0; o += nth) w0[o] = q.w[0][o];
  for (int o = tid; o < N1; o += nth) w1[o] = q.w[1][o];
  const T w2 = q.w[2][o2];
  T* slot = out + (int64_t)pid * Q::TS + (int64_t)o2 * N0 * N1;
  staged_copy<T, BIG_AC_THREADS, N0 * N1>([&](int e) { return slot[e]; },
                                       [&](int e, T v) { const int o1 = e / N0; pl[o1 * PT + e - o1 * N0] = v; });
  __syncthreads();
  mfma_lines_cols<T, N1>(pl, N0, 1, PT, q.ST[1]);
  __syncthreads();
  mfma_lines_cols<T, N0>(pl, N1, PT, 1, q.ST[0]);
  __syncthreads();
  staged_copy<T, BIG_AC_THREADS, N0 * N1>(
      [&](int e) {
        const int o1 = e / N0, o0 = e - o1 * N0;
        return w0[o0] * w1[o1] * w2 * pl[o1 * PT + o0];
      },
      [&](int e, T v) { slot[e] = v; });
}

template <class T, int NA, int NL, int ND>
void fdm_big_launch_nd(const LevelDev<T>& L, const T* r, T* out, int npx, int npy, int npz, hipStream_t s) {
  using Q = BigPatch<T, NA, NL, ND>;
  const int npatch = npx * npy * npz;
  hipLaunchKernelGGL((fdm_big_a<T, NA, NL, ND>), dim3(xcd_grid(npatch * Q::L2)), dim3(BIG_AC_THREADS), 0, s, L, r,
                     out, npx, npy, npz);
  // stage B contracts only along direction 2: one wave per output column block
  // (3 for length 43: a fourth wave would idle through both passes)
  constexpr int thb = big_b_threads<Q::L2>();
  hipLaunchKernelGGL((fdm_big_b<T, NA, NL, ND>), dim3(xcd_grid(npatch * Q::L1)), dim3(thb), 0, s, L, out, npx,
                     npy, npz);
  hipLaunchKernelGGL((fdm_big_c<T, NA, NL, ND>), dim3(xcd_grid(npatch * Q::L2)), dim3(BIG_AC_THREADS), 0, s, L,
                     out, npx, npy, npz);
}

template <class T, int NA, int NL>
int fdm_big_launch(const LevelDev<T>& L, int nd, const T* r, T* out, int npx, int npy, int npz, hipStream_t s) {
  if (nd < 0) {
    if constexpr (NA == NL) {
      fdm_big_launch_nd<T, NA, NL, -1>(L, r, out, npx, npy, npz, s);
      return 0;
    }
    return -4;
  }
  if (nd == 0) fdm_big_launch_nd<T, NA, NL, 0>(L, r, out, npx, npy, npz, s);
  else if (nd == 1) fdm_big_launch_nd<T, NA, NL, 1>(L, r, out, npx, npy, npz, s);
  else fdm_big_launch_nd<T, NA, NL, 2>(L, r, out, npx, npy, npz, s);
  return 0;
}

}  // namespace dgmg

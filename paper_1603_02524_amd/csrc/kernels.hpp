// HIP kernels for gfx950 (MI355X): sum-factorised DG operator, Schwarz patch
// solves by fast diagonalisation, deterministic overlap summation, p-transfers.
//
// Vector layout (all kernels): element-major, element e = m1 + N1 (m2 + N2 m3),
// local node (k NP + j) NP + i, direction 1 fastest.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgmg {

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }
constexpr int imax(int a, int b) { return a > b ? a : b; }
constexpr int imin(int a, int b) { return a < b ? a : b; }
constexpr int round64(int a) { return (a + 63) / 64 * 64; }

constexpr int NUM_XCD = 8;  // MI355X: 8 accelerator complex dies, blocks dispatched round-robin

// Logical block index such that each XCD receives one contiguous range of
// logical blocks (neighbouring elements then share that XCD's L2).  The grid
// is launched with NUM_XCD * ceil(G / NUM_XCD) blocks; returns -1 for padding.
__device__ __forceinline__ int xcd_block(int G) {
  const int per = (G + NUM_XCD - 1) / NUM_XCD;
  const int b = blockIdx.x;
  const int lb = (b % NUM_XCD) * per + b / NUM_XCD;
  return lb < G ? lb : -1;
}
inline int xcd_grid(int G) { return NUM_XCD * ((G + NUM_XCD - 1) / NUM_XCD); }

enum { ECOEF_N = 8, E_TWO_DX = 0, E_HALF_DX, E_CL, E_CNL, E_BL, E_CR, E_CNR, E_BR };

template <class T>
struct DirDev {
  int N = 1, periodic = 0;
  int nl = 0;  // continuous levels: stored lattice nodes of the direction
  int n_ec = 0, n_fc = 0, nf = 0;
  const T* ecoef = nullptr;  // N * 8 (see ECOEF enum)
  const int* nbr = nullptr;  // N * 2
  const T* S_ec = nullptr;   // N * n_ec^2, row-major S[k][j]
  const T* ST_ec = nullptr;  // the transposes
  const T* lam_ec = nullptr;
  const T* w_ec = nullptr;
  const T* S_fc = nullptr;   // nf * n_fc^2
  const T* ST_fc = nullptr;
  const T* lam_fc = nullptr;
  const T* w_fc = nullptr;
  // offsets into the level vector of every patch position (-1 outside a
  // Dirichlet domain): N * n_ec and nf * n_fc
  const int* goff_ec = nullptr;
  const int* goff_fc = nullptr;
};

template <class T>
struct LevelDev {
  int dim = 3, P = 1, NP = 2, NO = 0, NPc = 0;
  int se = 0;  // 1: continuous spectral-element level (lattice vectors)
  int n_elem = 0;
  int64_t n_dof = 0;
  const T* Ls = nullptr;   // NP*NP
  const T* D = nullptr;    // NP*NP, D[i*NP+k] = phi_k'(eta_i)
  const T* rho = nullptr;  // NP
  const T* J = nullptr;    // NP x NPc interpolation from the coarser level
  const int* active = nullptr;  // batched solves: the kernels return at once when *active == 0
  DirDev<T> dir[3];
};

__device__ __forceinline__ bool inactive(const int* flag) { return flag != nullptr && *flag == 0; }

// Patches of one launch: per direction the patch indices start + stride * k,
// k = 0 .. count - 1 (the additive sweeps take all of them: start 0, stride 1;
// a colour class of the multiplicative smoothers takes every k-th).
struct PatchLat {
  int start[3] = {0, 0, 0};
  int stride[3] = {1, 1, 1};
};

// Work list of a batched launch: one kernel over the work of many grids.  The
// launch's logical blocks are split into consecutive ranges, range g
// (starts[g] <= b < starts[g + 1], g < ng) doing grid g's blocks with the
// arguments descs[g] (device arrays; the grid index is uniform per block, so
// these reads are scalar loads).
template <class A>
struct BatchList {
  const A* descs = nullptr;
  const int* starts = nullptr;
  int ng = 0;
};

// Arguments of logical block b of a batched launch, copied into the block's
// LDS slot `args` (the kernels index their argument structs with run-time
// direction indices: from LDS that stays a plain LDS read, from a local copy it
// would go through scratch memory); returns the block's index within its grid.
// Called by every thread of the block.
template <class A>
__device__ __forceinline__ int batch_pick(const BatchList<A>& bl, int b, A* args) {
  static_assert(sizeof(A) % sizeof(int) == 0, "argument struct of whole words");
  const int* __restrict__ st = bl.starts;
  int lo = 0, hi = bl.ng - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (st[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  const int* __restrict__ src = reinterpret_cast<const int*>(bl.descs + lo);
  int* dst = reinterpret_cast<int*>(args);
  for (int i = threadIdx.x; i < (int)(sizeof(A) / sizeof(int)); i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  return b - st[lo];
}

// ---------------------------------------------------------------- block reduction
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic block sum (fixed shuffle tree then fixed order over waves).
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
  }
  return s;  // valid in thread 0
}

// ================================================================ operator apply
// y = A x (MODE 0), y = f - A x (MODE 1), y = A x plus per-block partial x.y (MODE 2),
// or the restriction of f - A x to the next coarser level, y = (J^T x J^T x J^T)(f - A x)
// per element (MODE 3: the V-cycle's residual and restriction in one pass; the
// fine residual stays in LDS and the transfer's contraction passes run on it).
// One thread owns one line of one element in one direction, and the lines of
// all directions run at once (their global loads overlap instead of forming
// one latency chain per direction).  Each node receives exactly one
// contribution per direction, stored in that direction's LDS tile; the tiles
// are summed in direction order at the end.  Neighbour traces and normal
// derivatives are read from the neighbour's line (eq. (L:generic)).
// Elements per block: lines of all directions fill about DGMG_APPLY_LINES threads.
#ifndef DGMG_APPLY_LINES
#define DGMG_APPLY_LINES 256
#endif
// Rows of the line product unrolled together (independent accumulation chains).
#ifndef DGMG_APPLY_ROWS
#define DGMG_APPLY_ROWS 1
#endif
template <int NP, int DIM>
constexpr int apply_epb() {
  return imax(1, DGMG_APPLY_LINES / (DIM * ipow(NP, DIM - 1)));
}
template <int NP, int DIM>
constexpr int apply_threads() {
  return imin(1024, round64(apply_epb<NP, DIM>() * DIM * ipow(NP, DIM - 1)));
}

// A kernel-argument pointer pinned in scalar registers: selecting between such
// values per lane stays a register select instead of becoming a per-lane load
// from the argument segment (which would make the loads behind it dependent).
template <class P>
__device__ __forceinline__ P* sgpr_ptr(P* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<P*>(((uint64_t)hi << 32) | lo);
}

// Move n <= N values with every load of a thread issued before any of its
// stores (a plain strided loop waits for each load before the next one
// starts).  NT is the block size; ld(e) reads element e (called with e < n
// only), st(e, v) writes it.
template <class T, int NT, int N, class Ld, class St>
__device__ __forceinline__ void staged_copy(Ld ld, St st, int n = N) {
  constexpr int C = (N + NT - 1) / NT;
  const int tid = threadIdx.x;
  T v[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int e = tid + c * NT;
    v[c] = ld(e < n ? e : n - 1);
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int e = tid + c * NT;
    if (e < n) st(e, v[c]);
  }
}

// Own elements staged in LDS (coalesced loads) when the tiles are small: the
// lines of the block's own elements are then read from LDS and only the
// neighbours' lines from global memory.  A line along direction 0 is contiguous,
// so the lanes of a wave (one line each) are NP values apart and a load touches
// about one cache line per lane: staging removes the costliest third of the line
// loads.
template <int NP, int DIM>
constexpr bool apply_stage_own() {
  return NP <= 9 && apply_epb<NP, DIM>() * DIM * ipow(NP, DIM - 1) <= 1024;
}
template <class T, int DIM, int NP>
constexpr size_t apply_shmem() {
  return (size_t)(DIM + (apply_stage_own<NP, DIM>() ? 1 : 0)) * apply_epb<NP, DIM>() * ipow(NP, DIM) * sizeof(T);
}

// Everything one line needs besides its own values: indices, the neighbours'
// lines (masks ml, mr), the face coefficients and the mass factor.
template <class T, int NP>
struct ApplyLine {
  int d, el, base, stride;
  T ml, mr, mo;
  T c_two_dx, c_cl, c_cnl, c_bl, c_cr, c_cnr, c_br;
  T wlv[NP], wrv[NP];
};

template <class T, int DIM, int NIN, int NOUT, int NEF, int D, bool RESTRICT, int NPC>
__device__ __forceinline__ void xfer_pass(const T* __restrict__ sJ, const T* __restrict__ src,
                                          T* __restrict__ dst, int ne);

template <class T>
struct ApplyArgs {
  LevelDev<T> L;
  const T* x = nullptr;
  const T* f = nullptr;
  T* y = nullptr;
  double* part = nullptr;
  int nblk = 0;
};

// BATCH: the arguments come from the work list bl (ntot logical blocks in all)
template <class T, int DIM, int NP, int MODE, bool BATCH = false>
__global__ void __launch_bounds__(1024) apply_kernel(ApplyArgs<T> a0, BatchList<ApplyArgs<T>> bl, int ntot) {
  constexpr int NE = ipow(NP, DIM), NLN = ipow(NP, DIM - 1), EPB = apply_epb<NP, DIM>();
  constexpr int P = NP - 1;
  constexpr bool STAGE = apply_stage_own<NP, DIM>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // per-direction contribution tiles, then (STAGE) the block's own elements
  T* sy = reinterpret_cast<T*>(smem_raw);
  T* sx = sy + DIM * EPB * NE;
  __shared__ double red[16];
  __shared__ __align__(16) int sargs_raw[BATCH ? sizeof(ApplyArgs<T>) / sizeof(int) : 1];
  ApplyArgs<T>* sargs = reinterpret_cast<ApplyArgs<T>*>(sargs_raw);
  const ApplyArgs<T>* ap;
  int blk;
  if constexpr (BATCH) {
    const int b = xcd_block(ntot);
    if (b < 0) return;
    blk = batch_pick(bl, b, sargs);
    ap = sargs;
  } else {
    blk = xcd_block(a0.nblk);
    if (blk < 0) return;
    ap = &a0;
  }
  const LevelDev<T>& L = ap->L;
  const T* __restrict__ x = ap->x;
  const T* __restrict__ f = ap->f;
  T* __restrict__ y = ap->y;
  double* __restrict__ part = ap->part;
  if (inactive(L.active)) return;
  const int e0 = blk * EPB;
  const int ne = imin(EPB, L.n_elem - e0);
  const int tid = threadIdx.x, nth = blockDim.x;
  const int64_t g0 = (int64_t)e0 * NE;
  const int N1 = L.dir[0].N, N2 = L.dir[1].N;
  // stiffness matrix rows: uniform addresses in the constant address space,
  // so the row loop reads them with scalar loads into SGPR operands; rows
  // longer than 72 bytes (2D, large P) would not fit the scalar registers and
  // are staged in LDS instead (uniform-address reads)
  constexpr bool SLS = NP * sizeof(T) <= 72;
  __shared__ T sLsL[SLS ? 1 : NP * NP];
  if constexpr (!SLS) {
    for (int q = tid; q < NP * NP; q += nth) sLsL[q] = L.Ls[q];
    __syncthreads();
  }
  // MODE 3: the interpolation matrix J (NP x NPC, row-major) of the restriction
  constexpr int NPC = (NP - 1) / 2 + 1;  // N_P of the next coarser level, P_c = floor(P / 2)
  static_assert(MODE != 3 || STAGE, "the fused restriction needs the own-element LDS buffer");
  __shared__ T sJx[MODE == 3 ? NP * NPC : 1];
  if constexpr (MODE == 3)
    for (int q = tid; q < NP * NPC; q += nth) sJx[q] = L.J[q];
  using CT = const __attribute__((address_space(4))) T;
  CT* __restrict__ Ls = (CT*)L.Ls;
  CT* __restrict__ D0 = (CT*)L.D;
  CT* __restrict__ DP = (CT*)(L.D + P * NP);
  const T* __restrict__ rho = L.rho;
  const int per_dir = ne * NLN;
  // per-direction kernel arguments in scalar registers; the per-lane choice
  // below is arithmetic with 0/1 flags (a select chain over them gets turned
  // into a small scratch array or into per-lane loads of the arguments)
  using GT = const __attribute__((address_space(1))) T;  // global memory
  GT* ec0 = (GT*)sgpr_ptr(L.dir[0].ecoef);
  GT* ec1 = (GT*)sgpr_ptr(L.dir[1].ecoef);
  GT* ec2 = (GT*)sgpr_ptr(L.dir[DIM - 1].ecoef);
  const int64_t eo1 = ec1 - ec0, eo2 = ec2 - ec0;
  const int per0 = __builtin_amdgcn_readfirstlane(L.dir[0].periodic);
  const int per1 = __builtin_amdgcn_readfirstlane(L.dir[1].periodic);
  const int per2 = __builtin_amdgcn_readfirstlane(L.dir[DIM - 1].periodic);
  const int N3 = __builtin_amdgcn_readfirstlane(L.dir[DIM - 1].N);
  // The vector the epilogue reads besides the tiles (f for the residual, x for
  // the dot product) is fetched now, so that its latency overlaps the line work
  // (launches use apply_threads() threads, so FQ values per thread cover the block).
  constexpr int TH = apply_threads<NP, DIM>(), FQ = (EPB * NE + TH - 1) / TH;
  constexpr bool PREF = MODE != 0 && NP <= 9;
  T pre[PREF ? FQ : 1];
  if constexpr (PREF) {
    const T* __restrict__ src = (MODE == 1 || MODE == 3) ? f : x;
#pragma unroll
    for (int j = 0; j < FQ; ++j) {
      const int q = tid + j * nth;
      pre[j] = q < ne * NE ? src[g0 + q] : T(0);
    }
  }
  // Loads of line q (all issued as one group): neighbours' lines (unconditional
  // loads at a valid address, masked later), coefficients, mass factors and,
  // unless staged, the own line into v.
  auto prep = [&](int q, ApplyLine<T, NP>& A, T* v, bool own) {
    const int d = q / per_dir;
    const int ln = q - d * per_dir;
    const int el = ln / NLN, t = ln - el * NLN;
    const int e = e0 + el;
    int m[3];
    m[0] = e % N1;
    m[1] = DIM == 3 ? (e / N1) % N2 : e / N1;
    m[2] = DIM == 3 ? e / (N1 * N2) : 0;
    // per-direction fields chosen per lane (the direction varies inside a wave)
    const int f0 = d == 0, f1 = d == 1, f2 = d == 2;
    const int md = f0 * m[0] + f1 * m[1] + f2 * m[2];
    const int Nd = f0 * N1 + f1 * N2 + f2 * N3;
    const int perd = f0 * per0 + f1 * per1 + f2 * per2;
    GT* __restrict__ ecoef = ec0 + (f1 * eo1 + f2 * eo2);
    const int estride = f0 + f1 * N1 + f2 * (N1 * N2);
    // line base and stride inside the element; indices of the other directions
    const int ia = t % NP, ib = t / NP;  // local indices of the other directions (in order)
    int base, stride;
    if (d == 0) {
      base = t * NP; stride = 1;
    } else if (d == 1) {
      base = ia + ib * NP * NP; stride = NP;
    } else {
      base = t; stride = NP * NP;
    }
    A.d = d;
    A.el = el;
    A.base = base;
    A.stride = stride;
    // neighbours along d: m -/+ 1, wrapped when periodic, none (-1) at a
    // Dirichlet end (the element neighbour table of the setup, computed here so
    // that no load depends on another)
    const int nl = md > 0 ? md - 1 : (perd ? Nd - 1 : -1);
    const int nr = md < Nd - 1 ? md + 1 : (perd ? 0 : -1);
    A.ml = nl >= 0 ? T(1) : T(0);
    A.mr = nr >= 0 ? T(1) : T(0);
    if (own) {
#pragma unroll
      for (int k = 0; k < NP; ++k) v[k] = x[g0 + el * NE + base + k * stride];
    }
    GT* c = ecoef + md * ECOEF_N;
    A.c_two_dx = c[E_TWO_DX];
    A.c_cl = c[E_CL];
    A.c_cnl = c[E_CNL];
    A.c_bl = c[E_BL];
    A.c_cr = c[E_CR];
    A.c_cnr = c[E_CNR];
    A.c_br = c[E_BR];
    const T ra = rho[ia], rb = DIM == 3 ? rho[ib] : T(1);
    T ha, hb;  // half element sizes of the other directions
    if (DIM == 2) {
      ha = d == 0 ? ec1[m[1] * ECOEF_N + E_HALF_DX] : ec0[m[0] * ECOEF_N + E_HALF_DX];
      hb = T(1);
    } else {
      const T h0 = ec0[m[0] * ECOEF_N + E_HALF_DX];
      const T h1 = ec1[m[1] * ECOEF_N + E_HALF_DX];
      const T h2 = ec2[m[2] * ECOEF_N + E_HALF_DX];
      ha = d == 0 ? h1 : h0;
      hb = d == 2 ? h1 : h2;
    }
    // mass factor of the other directions at this line
    A.mo = DIM == 2 ? ha * ra : ha * ra * hb * rb;
    const T* wl = x + (int64_t)(e + (nl >= 0 ? nl - md : 0) * estride) * NE + base;
    const T* wr = x + (int64_t)(e + (nr >= 0 ? nr - md : 0) * estride) * NE + base;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      A.wlv[k] = wl[k * stride];
      A.wrv[k] = wr[k * stride];
    }
  };
  // the line's contribution mo * (L_d-row terms) into its direction's tile
  auto finish = [&](const ApplyLine<T, NP>& A, const T* v) {
    T d0 = 0, dP = 0, dL = 0, dR = 0;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      d0 += D0[k] * v[k];
      dP += DP[k] * v[k];
      dL += DP[k] * A.wlv[k];
      dR += D0[k] * A.wrv[k];
    }
    const T uL = A.ml * A.wlv[P], uR = A.mr * A.wrv[0];
    dL *= A.ml;
    dR *= A.mr;
    const T jl = v[0] - uL, jr = v[P] - uR;
    const T fl = A.c_cl * d0 + A.c_cnl * dL + A.c_bl * jl;
    const T fr = -A.c_cr * dP - A.c_cnr * dR + A.c_br * jr;
    const T cl = A.c_cl * jl, cr = A.c_cr * jr, tdx = A.c_two_dx;
    T* __restrict__ syd = sy + (A.d * ne + A.el) * NE + A.base;
#pragma unroll DGMG_APPLY_ROWS  // a few rows of Ls live at a time (registers for the line data)
    for (int i = 0; i < NP; ++i) {
      T s = 0;
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        if constexpr (SLS) s += Ls[__builtin_amdgcn_readfirstlane(i) * NP + k] * v[k];
        else s += sLsL[i * NP + k] * v[k];
      }
      const int iu = __builtin_amdgcn_readfirstlane(i);
      T o = tdx * s + cl * D0[iu] - cr * DP[iu];
      if (i == 0) o += fl;
      if (i == P) o += fr;
      syd[i * A.stride] = A.mo * o;
    }
  };
  if constexpr (STAGE) {
    // one line per thread (the launch covers all lines of the block)
    constexpr int SQ = (EPB * NE + TH - 1) / TH;
    T st[SQ];
#pragma unroll
    for (int j = 0; j < SQ; ++j) {
      const int q = tid + j * nth;
      st[j] = q < ne * NE ? x[g0 + q] : T(0);
    }
    const bool has = tid < DIM * per_dir;
    ApplyLine<T, NP> A;
    T v[NP];
    prep(has ? tid : 0, A, v, false);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < SQ; ++j) {
      const int q = tid + j * nth;
      if (q < ne * NE) sx[q] = st[j];
    }
    __syncthreads();
    if (has) {
#pragma unroll
      for (int k = 0; k < NP; ++k) v[k] = sx[A.el * NE + A.base + k * A.stride];
      finish(A, v);
    }
  } else {
    for (int q = tid; q < DIM * per_dir; q += nth) {
      ApplyLine<T, NP> A;
      T v[NP];
      prep(q, A, v, true);
      if constexpr (NP <= 9) __builtin_amdgcn_sched_barrier(0);
      finish(A, v);
    }
  }
  __syncthreads();
  double acc = 0.0;
  const int dstride = ne * NE;
  auto out = [&](int q, T other) {
    T val = sy[q] + sy[dstride + q];
    if (DIM == 3) val += sy[2 * dstride + q];
    if (MODE == 0) {
      y[g0 + q] = val;
    } else if (MODE == 1) {
      y[g0 + q] = other - val;
    } else if (MODE == 3) {
      sx[q] = other - val;  // the own elements' x are no longer needed
    } else {
      y[g0 + q] = val;
      acc += (double)other * (double)val;
    }
  };
  if constexpr (PREF) {
#pragma unroll
    for (int j = 0; j < FQ; ++j) {
      const int q = tid + j * nth;
      if (q < ne * NE) out(q, pre[j]);
    }
  } else if constexpr (MODE == 0) {
    for (int q = tid; q < ne * NE; q += nth) out(q, T(0));
  } else {
    // every load of f (x) issued before the sums that use them
    const T* __restrict__ src = (MODE == 1 || MODE == 3) ? f : x;
    staged_copy<T, TH, EPB * NE>([&](int q) { return src[g0 + q]; }, [&](int q, T v) { out(q, v); }, ne * NE);
  }
  if (MODE == 2) {
    const double s = block_sum(acc, red);
    if (tid == 0) part[blk] = s;
  }
  if constexpr (MODE == 3) {
    // the transfer kernel's restriction passes, on the residual in LDS (the
    // direction tiles serve as the two pass buffers); y is the coarse vector
    constexpr int NEC = ipow(NPC, DIM);
    __syncthreads();
    T* bA = sy;
    T* bB = sy + EPB * NE;
    xfer_pass<T, DIM, NP, NPC, NE, 0, true, NPC>(sJx, sx, bA, ne);
    __syncthreads();
    xfer_pass<T, DIM, NP, NPC, NE, 1, true, NPC>(sJx, bA, bB, ne);
    __syncthreads();
    const T* res = bB;
    if constexpr (DIM == 3) {
      xfer_pass<T, DIM, NP, NPC, NE, 2, true, NPC>(sJx, bB, bA, ne);
      __syncthreads();
      res = bA;
    }
    T* yc = y + (int64_t)e0 * NEC;
    for (int q = tid; q < ne * NEC; q += nth) {
      const int el = q / NEC;
      yc[q] = res[el * NE + q - el * NEC];
    }
  }
}

template <class T, int DIM, int NP, int MODE, bool BATCH>
void apply_go(const ApplyArgs<T>& a, const BatchList<ApplyArgs<T>>& bl, int nlog, hipStream_t s) {
  constexpr int TH = apply_threads<NP, DIM>();
  const size_t shm = apply_shmem<T, DIM, NP>();
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)apply_kernel<T, DIM, NP, MODE, BATCH>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipLaunchKernelGGL((apply_kernel<T, DIM, NP, MODE, BATCH>), dim3(xcd_grid(nlog)), dim3(TH), shm, s, a, bl, nlog);
}

// Blocks of one grid's apply: groups of apply_epb elements.
template <int DIM, int NP>
int apply_blocks(int n_elem) {
  constexpr int EPB = apply_epb<NP, DIM>();
  return (n_elem + EPB - 1) / EPB;
}

// The fused residual + restriction (mode 3) is built where the own elements are
// staged in LDS and the coarse level's order follows P_c = floor(P / 2).
template <class T, int DIM, int NP>
bool apply_mode3_ok(const LevelDev<T>& L) {
  if constexpr (apply_stage_own<NP, DIM>()) return L.NPc == (NP - 1) / 2 + 1 && L.J != nullptr;
  return false;
}

template <class T, int DIM, int NP, bool BATCH>
int apply_mode(int mode, const ApplyArgs<T>& a, const BatchList<ApplyArgs<T>>& bl, int nlog, hipStream_t s) {
  if (mode == 0) apply_go<T, DIM, NP, 0, BATCH>(a, bl, nlog, s);
  else if (mode == 1) apply_go<T, DIM, NP, 1, BATCH>(a, bl, nlog, s);
  else if (mode == 2) apply_go<T, DIM, NP, 2, BATCH>(a, bl, nlog, s);
  else if constexpr (apply_stage_own<NP, DIM>()) apply_go<T, DIM, NP, 3, BATCH>(a, bl, nlog, s);
  else return -4;
  return 0;
}

template <class T, int DIM, int NP>
int apply_launch(const LevelDev<T>& L, int mode, const T* x, const T* f, T* y, double* part,
                 int* nblk_out, hipStream_t s) {
  const int nblk = apply_blocks<DIM, NP>(L.n_elem);
  if (nblk_out) *nblk_out = nblk;
  // fused residual + restriction: otherwise the caller runs the two steps
  if (mode == 3 && !apply_mode3_ok<T, DIM, NP>(L)) return -4;
  ApplyArgs<T> a;
  a.L = L;
  a.x = x;
  a.f = f;
  a.y = y;
  a.part = part;
  a.nblk = nblk;
  return apply_mode<T, DIM, NP, false>(mode, a, BatchList<ApplyArgs<T>>{}, nblk, s);
}

// One launch over the applies of many grids (same NP and mode): ntot logical
// blocks, grid g's apply_blocks in the range of bl.
template <class T, int DIM, int NP>
int apply_batch_launch(int mode, const BatchList<ApplyArgs<T>>& bl, int ntot, hipStream_t s) {
  return apply_mode<T, DIM, NP, true>(mode, ApplyArgs<T>{}, bl, ntot, s);
}

// ================================================================ FDM patch solve
// Patch-solve code choices: the eigenvalue scaling by reciprocal estimate and
// Newton steps instead of IEEE division, and for rows exactly 16 long the
// gather / scatter in 16-lane row groups (no index division, per-column table
// values in registers).
#ifndef DGMG_FDM_DIV_NR
#define DGMG_FDM_DIV_NR 1
#endif
#ifndef DGMG_FDM_GATHER2D
#define DGMG_FDM_GATHER2D 1
#endif
// Matrix operands of consecutive passes in two register sets used in turn
// (the next pass's matrix loads while the current pass runs).
#ifndef DGMG_FDM_PING
#define DGMG_FDM_PING 1
#endif
// FP64: the forward and backward passes of tile dimension 2 fused (the scaled
// forward results feed the backward product from registers).
#ifndef DGMG_FDM_FUSE2
#define DGMG_FDM_FUSE2 1
#endif

// v / d for d > 0 of moderate magnitude (sums of patch eigenvalues): hardware
// reciprocal estimate, Newton-Raphson refinement of 1/d, then one residual
// correction of the quotient (within an ulp or two of the rounded quotient).
__device__ __forceinline__ double div_nr(double v, double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  r = fma(fma(-d, r, 1.0), r, r);
  const double q = v * r;
  return fma(fma(-d, q, v), r, q);
}
__device__ __forceinline__ float div_nr(float v, float d) {
  float r = __builtin_amdgcn_rcpf(d);
  r = fmaf(fmaf(-d, r, 1.0f), r, r);
  const float q = v * r;
  return fmaf(fmaf(-d, q, v), r, q);
}
// One patch per block.  The LDS tile keeps the normal direction fastest:
// tile[(l2 * NL + l1) * NAP + a], NAP = NA rounded up to an odd pitch so that
// the lines of the fastest pass spread over the LDS banks.  NA = 2P for a
// face-centred patch (the element-centred size otherwise), NL = NP + 2 N_O.
// Each contraction pass runs on the matrix cores: the lines of the tile are the
// M dimension (blocks of 16), the 1D eigenbasis is the B operand held in
// registers, and each wave overwrites its line blocks in place.
template <int NA, int NL, int DIM>
constexpr int fdm_tile() {
  return NA * ipow(NL, DIM - 1);
}
template <int NA>
constexpr int fdm_pitch() {
  return NA % 2 == 0 ? NA + 1 : NA;
}
template <int NA, int NL, int DIM>
constexpr int fdm_tile_padded() {
  return fdm_pitch<NA>() * ipow(NL, DIM - 1);
}
// Lines up to this length are contracted on the VALU, longer ones on the
// matrix cores (fdm_pass_any).
#ifndef DGMG_FDM_VALU_MAXLEN
#define DGMG_FDM_VALU_MAXLEN 9
#endif
// Default block size of a patch solve (the autotuner may choose another): a
// thread per line of the longest pass, at most 256; 3D tiles whose passes all
// run on the matrix cores take 4 waves, the size the autotuner picks for them
// (16 x 13 x 13, 13^3, 11^3 in FP64 and FP32).
template <int NA, int NL, int DIM>
constexpr int fdm_threads() {
  if (DIM == 3 && NA > DGMG_FDM_VALU_MAXLEN && NL > DGMG_FDM_VALU_MAXLEN) return 256;
  return imin(256, round64(imax(ipow(NL, DIM - 1), NA * ipow(NL, DIM - 2))));
}
template <class T, int NA, int NL, int DIM>
constexpr size_t fdm_shmem() {
  return (size_t)fdm_tile_padded<NA, NL, DIM>() * sizeof(T);
}

// Whole LDS of one patch-solve block: the tile plus the per-direction and
// per-row tables (largest over the sweep kinds) and some slack.
template <class T, int NA, int NL, int DIM>
constexpr size_t fdm_lds_total() {
  constexpr int NMAX = imax(NA, NL);
  constexpr int NROW = DIM == 3 ? imax(NL * NL, NA * NL) : imax(NL, NA);
  return fdm_shmem<T, NA, NL, DIM>() + 3 * NMAX * (sizeof(int) + 2 * sizeof(T)) +
         NROW * (2 * sizeof(int) + sizeof(T)) + 512;
}

// 16x16x4 matrix-core contraction (v_mfma_{f64,f32}_16x16x4): A[i][k] comes from lane
// i + 16k and B[k][j] from lane j + 16k.  Result register r of lane l holds
// D[row(l / 16, r)][l % 16] with row = l/16 + 4r for f64 and 4 (l/16) + r for f32
// (layouts checked on gfx950 with one-hot operands).
template <class T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};
template <>
struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

// Line start inside the padded tile for contraction dimension TD.
template <int NA, int NL, int TD>
__device__ __forceinline__ int fdm_line_base(int line) {
  constexpr int NAP = fdm_pitch<NA>();
  if (TD == 0) return line * NAP;
  const int a = line % NA, q = line / NA;
  return TD == 1 ? q * NAP * NL + a : q * NAP + a;
}

// The 1D matrix of a contraction (row-major LEN x LEN) in registers: lane
// (li, lk) = (lane % 16, lane / 16) holds B[4 ks + lk][16 nb + li], i.e. the
// A operand (B^T)[16 nb + li][4 ks + lk] of the transposed product.
template <class T, int LEN>
struct BOp {
  static constexpr int KS = (LEN + 3) / 4, NB = (LEN + 15) / 16;
  T b[NB][KS];
  // the matrix of another length with the same register shape (KS, NB)
  template <int LEN2>
  __device__ __forceinline__ void load_as(const T* __restrict__ Bm) {
    static_assert((LEN2 + 3) / 4 == KS && (LEN2 + 15) / 16 == NB, "register shapes differ");
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int k = 4 * ks + lk, j = nb * 16 + li;
        const T v = Bm[imin(k, LEN2 - 1) * LEN2 + imin(j, LEN2 - 1)];
        b[nb][ks] = (k < LEN2 && j < LEN2) ? v : T(0);
      }
  }
  __device__ __forceinline__ void load(const T* __restrict__ Bm) {
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int k = 4 * ks + lk, j = nb * 16 + li;
        // unconditional load at a valid index, zero outside the matrix (no branch)
        const T v = Bm[imin(k, LEN - 1) * LEN + imin(j, LEN - 1)];
        b[nb][ks] = (k < LEN && j < LEN) ? v : T(0);
      }
  }
};

// One contraction pass over tile dimension TD: every line v (length LEN) is
// replaced by B^T v, i.e. out_j = sum_k B[k][j] v_k.  The lines form the M
// dimension in blocks of 16; each wave owns whole blocks, reading a block
// (A operand) completely before writing it back in place.
struct NoPost {
  template <class T>
  __device__ __forceinline__ T operator()(int, int, T v) const { return v; }
};

// post(line, j, value) maps each result before it is stored (e.g. the
// eigenvalue scaling fused into the last forward pass).
// No lane-dependent branches: loads past the end of a line or of the line set
// read a valid element instead (the matrix operand is zero for k >= LEN, and
// results of lines past the set are discarded), and stores of rows j >= LEN or
// of lines past the set go to the lane's slot of `trash` (64 values, dead
// storage) instead of being masked.
template <class T, int NA, int NL, int DIM, int TD, class Post = NoPost, int BLEN = (TD == 0 ? NA : NL),
          bool TAIL = false>
__device__ __forceinline__ void fdm_pass(T* __restrict__ tile, T* __restrict__ trash,
                                         const BOp<T, BLEN>& B, Post post = Post(),
                                         const T* __restrict__ tail = nullptr) {
  static_assert(BOp<T, BLEN>::KS == BOp<T, TD == 0 ? NA : NL>::KS &&
                    BOp<T, BLEN>::NB == BOp<T, TD == 0 ? NA : NL>::NB,
                "operand register shape");
  // Product D = B^T V^T: the A operand is B^T (held as B.b), the B operand the
  // lines; lane (li, lk) then owns output column li = its own line, rows
  // j = 16 nb + row(lk, r), so results go back along the line it loaded.
  constexpr int NAP = fdm_pitch<NA>();
  constexpr int LEN = TD == 0 ? NA : NL;
  constexpr int LINES = TD == 0 ? ipow(NL, DIM - 1) : NA * ipow(NL, DIM - 2);
  constexpr int STRIDE = TD == 0 ? 1 : (TD == 1 ? NAP : NAP * NL);
  constexpr int KS = BOp<T, LEN>::KS, NB = BOp<T, LEN>::NB, MB = (LINES + 15) / 16;
  using M = Mfma<T>;
  // the wave index is uniform over the wave: keeping it scalar makes the block
  // loop a scalar loop
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = blockDim.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  for (int mb = wave; mb < MB; mb += nw) {
    const int line = mb * 16 + li;
    const bool lv = line < LINES;
    const int lc = imin(line, LINES - 1);
    const int base = fdm_line_base<NA, NL, TD>(lc);
    typename M::acc_t acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = typename M::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < (TAIL ? KS - 1 : KS); ++ks) {
      const int k = imin(4 * ks + lk, LEN - 1);
      const T a = tile[base + k * STRIDE];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = M::op(B.b[nb][ks], a, acc[nb]);
    }
    if constexpr (TAIL) {
      // LEN = 4 (KS - 1) + 1: the last contraction index is alone in its group
      // of four, so it is added on the VALU as a rank-one update (tail = row
      // LEN - 1 of B in LDS) instead of a fourth product that is 3/4 padding
      const T at = tile[base + (LEN - 1) * STRIDE];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = imin(nb * 16 + M::row(lk, r), LEN - 1);
          acc[nb][r] = __builtin_fma(tail[j], at, acc[nb][r]);
        }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = nb * 16 + M::row(lk, r);
        const bool ok = lv && j < LEN;
        const int jc = imin(j, LEN - 1);
        T* dst = ok ? tile + base + jc * STRIDE : trash + lane;
        *dst = post(lc, jc, acc[nb][r]);
      }
  }
}

// The last forward and the first backward contraction of tile dimension 2
// in one pass (FP64, lines of 5 to 16): a line block's forward results,
// scaled by post(line, j, value), stay in registers as the operand of the
// backward product instead of going through the tile and a barrier.  The f64
// result layout makes this possible: lane (li, lk) ends the forward product
// holding rows j = lk + 4r of its line li, which are exactly the contraction
// indices k = 4 ks + lk (ks = r) it supplies to the next product.  Rows
// j >= LEN are set to 0 (the backward matrix is zero there as well).  TAIL
// as in fdm_pass, for both products (tail, tailb: the last rows of the
// forward and backward matrices).
template <int NA, int NL, int DIM, class Post, int BLEN, bool TAIL>
__device__ __forceinline__ void fdm_pass_fused2(double* __restrict__ tile, double* __restrict__ trash,
                                                const BOp<double, BLEN>& Bf, const BOp<double, BLEN>& Bb,
                                                Post post, const double* __restrict__ tail,
                                                const double* __restrict__ tailb) {
  using T = double;
  constexpr int TD = 2;
  constexpr int LEN = NL;
  constexpr int LINES = NA * ipow(NL, DIM - 2);
  constexpr int STRIDE = fdm_pitch<NA>() * NL;
  constexpr int KS = BOp<T, LEN>::KS, NB = BOp<T, LEN>::NB, MB = (LINES + 15) / 16;
  static_assert(DIM == 3 && NB == 1 && KS >= 2, "lines of 5 to 16 values");
  static_assert(BOp<T, BLEN>::KS == KS && BOp<T, BLEN>::NB == NB, "operand register shape");
  using M = Mfma<T>;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = blockDim.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  for (int mb = wave; mb < MB; mb += nw) {
    const int line = mb * 16 + li;
    const bool lv = line < LINES;
    const int lc = imin(line, LINES - 1);
    const int base = fdm_line_base<NA, NL, TD>(lc);
    typename M::acc_t acc = typename M::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < (TAIL ? KS - 1 : KS); ++ks) {
      const int k = imin(4 * ks + lk, LEN - 1);
      acc = M::op(Bf.b[0][ks], tile[base + k * STRIDE], acc);
    }
    if constexpr (TAIL) {
      const T at = tile[base + (LEN - 1) * STRIDE];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = imin(M::row(lk, r), LEN - 1);
        acc[r] = __builtin_fma(tail[j], at, acc[r]);
      }
    }
    typename M::acc_t out = typename M::acc_t{0, 0, 0, 0};
    T v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = M::row(lk, r);  // = 4 r + lk: the next product's contraction index
      const T sv = post(lc, imin(j, LEN - 1), acc[r]);
      v[r] = j < LEN ? sv : T(0);
    }
#pragma unroll
    for (int r = 0; r < (TAIL ? KS - 1 : KS); ++r) out = M::op(Bb.b[0][r], v[r], out);
    if constexpr (TAIL) {
      // the last contraction index LEN - 1 = 4 (KS - 1) + 0 is held by lane
      // (li, 0) in register KS - 1: broadcast it to the line's four lanes,
      // rank-one update
      const T at = __shfl(v[KS - 1], li, 64);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = imin(M::row(lk, r), LEN - 1);
        out[r] = __builtin_fma(tailb[j], at, out[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = M::row(lk, r);
      const bool ok = lv && j < LEN;
      const int jc = imin(j, LEN - 1);
      T* dst = ok ? tile + base + jc * STRIDE : trash + lane;
      *dst = out[r];
    }
  }
}

template <class T, int NA, int NL, int DIM, int TD, class Post = NoPost>
__device__ __forceinline__ void fdm_pass(T* __restrict__ tile, T* __restrict__ trash, const T* __restrict__ Bm,
                                         Post post = Post()) {
  BOp<T, TD == 0 ? NA : NL> B;
  B.load(Bm);
  fdm_pass<T, NA, NL, DIM, TD, Post>(tile, trash, B, post);
}

// VALU form of a contraction pass: one line per thread, out_j = sum_k B[k][j] v_k,
// reading BT = B^T (row-major, so the coefficients of one output are one
// contiguous row) through scalar loads: the matrix is uniform over the block.
// Exact line lengths: FP64 vector FMA and FP64 MFMA have the same peak rate on
// gfx950, and the matrix-core form pads lengths like 13 to 16 in both the K
// and N dimensions (66 % useful work), so short lateral lines are cheaper here.
// Same post(line, j, value) contract as fdm_pass.
// Rows of the matrix per step of the VALU pass: the largest divisor R of LEN
// with R LEN values within 32 FP64 (64 FP32) SGPR pairs / SGPRs.
template <class T, int LEN>
constexpr int fdm_valu_rows() {
  constexpr int cap = sizeof(T) == 8 ? 32 : 64;
  int best = 1;
  for (int r = 1; r <= LEN; ++r)
    if (LEN % r == 0 && r * LEN <= cap) best = r;
  return best;
}

template <class T, int NA, int NL, int DIM, int TD, class Post = NoPost>
__device__ __forceinline__ void fdm_pass_valu(T* __restrict__ tile, const T* __restrict__ BTm,
                                              Post post = Post()) {
  constexpr int NAP = fdm_pitch<NA>();
  constexpr int LEN = TD == 0 ? NA : NL;
  constexpr int LINES = TD == 0 ? ipow(NL, DIM - 1) : NA * ipow(NL, DIM - 2);
  constexpr int STRIDE = TD == 0 ? 1 : (TD == 1 ? NAP : NAP * NL);
  using CT = const __attribute__((address_space(4))) T;
  CT* __restrict__ BT = (CT*)BTm;
  constexpr int R = fdm_valu_rows<T, LEN>();
  for (int line = threadIdx.x; line < LINES; line += blockDim.x) {
    const int base = fdm_line_base<NA, NL, TD>(line);
    T v[LEN];
#pragma unroll
    for (int k = 0; k < LEN; ++k) v[k] = tile[base + k * STRIDE];
    // R rows of BT per step: R independent accumulation chains, one scalar
    // load group per step, at most 32 FP64 (64 FP32) matrix values in SGPRs
#pragma unroll 1
    for (int j0 = 0; j0 < LEN; j0 += R) {
      const int ju = __builtin_amdgcn_readfirstlane(j0);
      T acc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = 0;
#pragma unroll
      for (int k = 0; k < LEN; ++k)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] += BT[(ju + r) * LEN + k] * v[k];
#pragma unroll
      for (int r = 0; r < R; ++r) tile[base + (j0 + r) * STRIDE] = post(line, j0 + r, acc[r]);
    }
  }
}

// Contraction pass of tile dimension TD on the unit that suits its length:
// lines up to DGMG_FDM_VALU_MAXLEN long go to the VALU (the matrix-core form
// would pad a length-9 line to 12 x 16, 42 % useful work), longer ones to the
// matrix cores (measured on an MI355X: length 13 lateral passes on the VALU made
// the 16 x 13 x 13 patch solve 9 % slower, every pass on the VALU 35 %).
template <class T, int NA, int NL, int DIM, int TD, class Post = NoPost>
__device__ __forceinline__ void fdm_pass_any(T* __restrict__ tile, T* __restrict__ trash, const T* __restrict__ Bm,
                                             const T* __restrict__ BTm, Post post = Post()) {
  constexpr int LEN = TD == 0 ? NA : NL;
  constexpr bool VALU = LEN <= DGMG_FDM_VALU_MAXLEN;
  if constexpr (VALU) fdm_pass_valu<T, NA, NL, DIM, TD, Post>(tile, BTm, post);
  else fdm_pass<T, NA, NL, DIM, TD, Post>(tile, trash, Bm, post);
}

// Tile geometry of one sweep kind, all compile-time: ND = normal direction of a
// face-centred patch (-1: element-centred).  Grid-natural order has direction 0
// fastest with lengths L0, L1, L2; the LDS tile keeps the normal direction
// fastest: tile[(l2 NL + l1) NAP + a].
template <int DIM, int ND, int NA, int NL>
struct FdmShape {
  static constexpr int L0 = ND == 0 ? NA : NL;
  static constexpr int L1 = ND == 1 ? NA : NL;
  static constexpr int L2 = DIM == 3 ? (ND == 2 ? NA : NL) : 1;
  static constexpr int TS = L0 * L1 * L2;
  static constexpr int NROW = L1 * L2;  // rows of the grid-natural order (fixed o1, o2)
  static constexpr int NAP = fdm_pitch<NA>();
  // tile stride of direction 0 (the normal / fastest tile dimension unless ND > 0)
  static constexpr int C0 = ND <= 0 ? 1 : NAP;
  // grid direction of tile dimension t (t = 0: the normal / fastest one)
  static constexpr int gd(int t) {
    return ND <= 0 ? t : (t == 0 ? ND : (t <= ND ? t - 1 : t));
  }
  static __device__ __forceinline__ int tpos(int o0, int o1, int o2) {
    const int o[3] = {o0, o1, o2};
    return ((DIM == 3 ? o[gd(2)] * NL : 0) + o[gd(1)]) * NAP + o[gd(0)];
  }
  static __device__ __forceinline__ void split(int q, int& o0, int& o1, int& o2) {
    o0 = q % L0;
    const int rest = q / L0;
    o1 = DIM == 3 ? rest % L1 : rest;
    o2 = DIM == 3 ? rest / L1 : 0;
  }
};

// Minimum waves per SIMD asked of the compiler: 6 for the 16 x 13 x 13 tile
// (P = 8 face-centred patches), so that its register use stays within 80 and
// six 4-wave blocks fit a CU, as its LDS allows; no constraint otherwise.
template <int NA, int NL>
constexpr int fdm_min_waves() {
  return NA == 16 && NL == 13 ? 6 : 1;
}
template <class T>
struct FdmArgs {
  LevelDev<T> L;
  const T* r = nullptr;  // residual (level vector)
  T* out = nullptr;      // weighted corrections, one tile per patch of the launch
  int npx = 1, npy = 1, npz = 1;
  PatchLat lat;
};

// BATCH: the arguments come from the work list bl (ntot logical blocks in all)
template <class T, int DIM, int NA, int NL, int ND, bool BATCH = false>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(fdm_min_waves<NA, NL>()))) fdm_kernel(FdmArgs<T> a0, BatchList<FdmArgs<T>> bl, int ntot) {
  using S = FdmShape<DIM, ND, NA, NL>;
  constexpr int TS = S::TS;
  constexpr int NMAX = imax(NA, NL);
  constexpr int GU = 4;  // elements gathered per thread before their LDS stores (loads in flight)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);
  __shared__ int goff[3][NMAX];  // offsets into the level vector (< 2^31 unknowns), -1 outside
  __shared__ T wv[3][NMAX];
  __shared__ T lv[3][NMAX];
  // rowoff is dead once the gather is done: the contraction passes use it as
  // their store trash (64 values)
  __shared__ __align__(8) int rowoff[imax(S::NROW, 64 * (int)sizeof(T) / (int)sizeof(int))];
  __shared__ int rowpos[S::NROW];
  __shared__ __align__(16) int sargs_raw[BATCH ? sizeof(FdmArgs<T>) / sizeof(int) : 1];
  FdmArgs<T>* sargs = reinterpret_cast<FdmArgs<T>*>(sargs_raw);
  const FdmArgs<T>* ap;
  int pid;
  if constexpr (BATCH) {
    const int b = xcd_block(ntot);
    if (b < 0) return;
    pid = batch_pick(bl, b, sargs);
    ap = sargs;
  } else {
    pid = xcd_block(a0.npx * a0.npy * (DIM == 3 ? a0.npz : 1));
    if (pid < 0) return;
    ap = &a0;
  }
  const LevelDev<T>& L = ap->L;
  const T* __restrict__ r = ap->r;
  T* __restrict__ out = ap->out;
  const int npx = ap->npx, npy = ap->npy;
  const PatchLat& lat = ap->lat;
  if (inactive(L.active)) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  int p[3];
  p[0] = lat.start[0] + lat.stride[0] * (pid % npx);
  p[1] = lat.start[1] + lat.stride[1] * ((pid / npx) % npy);
  p[2] = DIM == 3 ? lat.start[2] + lat.stride[2] * (pid / (npx * npy)) : 0;
  const int* go[3] = {nullptr, nullptr, nullptr};
  const T* wg[3] = {nullptr, nullptr, nullptr};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const DirDev<T>& dd = L.dir[d];
    const bool fc = d == ND;
    const int len = fc ? NA : NL;
    go[d] = fc ? dd.goff_fc + p[d] * NA : dd.goff_ec + p[d] * NL;
    wg[d] = fc ? dd.w_fc + p[d] * NA : dd.w_ec + p[d] * NL;
    const T* lam = fc ? dd.lam_fc + p[d] * NA : dd.lam_ec + p[d] * NL;
    for (int o = tid; o < len; o += nth) {
      goff[d][o] = go[d][o];
      wv[d][o] = wg[d][o];
      lv[d][o] = lam[o];
    }
  }
  // per row (o1, o2) of the grid-natural order: its offset in the level vector
  // (-1 outside a Dirichlet domain) and its tile position (its weight w1 w2 is
  // formed from the per-direction tables at the scatter)
  for (int rw = tid; rw < S::NROW; rw += nth) {
    const int o1 = DIM == 3 ? rw % S::L1 : rw, o2 = DIM == 3 ? rw / S::L1 : 0;
    const int g1 = go[1][o1], g2 = DIM == 3 ? go[2][o2] : 0;
    rowoff[rw] = (g1 | g2) < 0 ? -1 : g1 + g2;
    rowpos[rw] = S::tpos(0, o1, o2);
  }
  // 1D matrices of each tile dimension: forward t_j = sum_k S_kj r_k uses S,
  // backward u_k = sum_j S_kj t_j uses S^T (both row-major)
  const T* fwd[3] = {nullptr, nullptr, nullptr};
  const T* bwd[3] = {nullptr, nullptr, nullptr};
#pragma unroll
  for (int t = 0; t < DIM; ++t) {
    const int d = S::gd(t);
    const DirDev<T>& dd = L.dir[d];
    if (d == ND) {
      fwd[t] = dd.S_fc + (int64_t)p[d] * NA * NA;
      bwd[t] = dd.ST_fc + (int64_t)p[d] * NA * NA;
    } else {
      fwd[t] = dd.S_ec + (int64_t)p[d] * NL * NL;
      bwd[t] = dd.ST_ec + (int64_t)p[d] * NL * NL;
    }
  }
  // two operand register sets used in turn (3D, every pass on the matrix cores,
  // both lengths with the same register shape)
  constexpr bool PING = DGMG_FDM_PING && DIM == 3 && NA > DGMG_FDM_VALU_MAXLEN &&
                        NL > DGMG_FDM_VALU_MAXLEN && BOp<T, NA>::KS == BOp<T, NL>::KS &&
                        BOp<T, NA>::NB == BOp<T, NL>::NB;
  BOp<T, NA> P, Q;
  // FP64 with lateral lines of at most 16: the dimension-2 passes fused
  constexpr bool FUSE2 = DGMG_FDM_FUSE2 && PING && sizeof(T) == 8 && NL <= 16;
  // FP64 lateral lines with NL = 1 (mod 4): the last row of each of their
  // four matrices in LDS for the rank-one tail of those passes (in FP32 the
  // 16x16x4 product costs half as much and the tail measured slower)
  constexpr bool TAILK = PING && NL % 4 == 1 && sizeof(T) == 8;
  __shared__ T sBt[TAILK ? 4 : 1][TAILK ? NL : 1];
  if constexpr (TAILK) {
    const T* rows[4] = {fwd[1], fwd[2], bwd[2], bwd[1]};
#pragma unroll
    for (int m = 0; m < 4; ++m)
      for (int j = tid; j < NL; j += nth) sBt[m][j] = rows[m][(NL - 1) * NL + j];
  }
  if constexpr (PING) P.load(fwd[0]);
  __syncthreads();
  // gather R_s r in grid-natural order (coalesced global reads); GU loads are
  // issued before their LDS stores; positions outside a Dirichlet domain read
  // r[0] and store 0
  constexpr bool G2D = DGMG_FDM_GATHER2D && S::L0 == 16;  // shorter rows would idle lanes (measured slower)
  if constexpr (G2D) {
    // lanes in groups of 16 along direction 0 (o0 = tid % 16), rows in steps of nth / 16
    const int o0 = tid & 15, rstep = nth >> 4;
    const bool colok = o0 < S::L0;
    const int oc = colok ? o0 : 0;
    const int g0 = goff[0][oc], pc = oc * S::C0;
    for (int rw0 = tid >> 4; rw0 < S::NROW; rw0 += GU * rstep) {
      T v[GU];
      int pos[GU];
#pragma unroll
      for (int u = 0; u < GU; ++u) {
        const int rw = rw0 + u * rstep;
        const bool in = colok && rw < S::NROW;
        const int rwc = rw < S::NROW ? rw : 0;
        const int ro = rowoff[rwc];
        const bool ok = in && (g0 | ro) >= 0;
        v[u] = r[ok ? g0 + ro : 0];
        v[u] = ok ? v[u] : T(0);
        pos[u] = in ? rowpos[rwc] + pc : -1;
      }
#pragma unroll
      for (int u = 0; u < GU; ++u)
        if (pos[u] >= 0) tile[pos[u]] = v[u];
    }
  } else {
    for (int q0 = tid; q0 < TS; q0 += GU * nth) {
      T v[GU];
      int pos[GU];
#pragma unroll
      for (int u = 0; u < GU; ++u) {
        const int q = q0 + u * nth;
        const int qq = q < TS ? q : 0;
        const int o0 = qq % S::L0, rw = qq / S::L0;
        const int g0 = goff[0][o0], ro = rowoff[rw];
        const bool ok = q < TS && (g0 | ro) >= 0;
        v[u] = r[ok ? g0 + ro : 0];
        v[u] = ok ? v[u] : T(0);
        pos[u] = q < TS ? rowpos[rw] + o0 * S::C0 : -1;
      }
#pragma unroll
      for (int u = 0; u < GU; ++u)
        if (pos[u] >= 0) tile[pos[u]] = v[u];
    }
  }
  __syncthreads();
  T* trash = reinterpret_cast<T*>(rowoff);
  // the last forward pass divides each result by the sum of the 1D eigenvalues
  // of its tile position: line = a + NA l1 (3D; a in 2D), j = l2 (3D; l1 in 2D)
  const auto scale = [&](int line, int j, T v) -> T {
    const int a = line % NA;
    T den = lv[S::gd(0)][a] + lv[S::gd(1)][DIM == 3 ? line / NA : j];
    if (DIM == 3) den += lv[S::gd(2)][j];
    if constexpr (DGMG_FDM_DIV_NR) return div_nr(v, den);
    else return v / den;
  };
  if constexpr (PING) {
    // every pass on the matrix cores with one register shape: the next pass's
    // matrix is loaded into the idle set while the current pass runs
    Q.template load_as<NL>(fwd[1]);
    fdm_pass<T, NA, NL, DIM, 0, NoPost, NA>(tile, trash, P);
    __syncthreads();
    P.template load_as<NL>(fwd[2]);
    fdm_pass<T, NA, NL, DIM, 1, NoPost, NA, TAILK>(tile, trash, Q, NoPost(), sBt[0]);
    __syncthreads();
    Q.template load_as<NL>(bwd[2]);
    if constexpr (FUSE2) {
      // forward and backward along dimension 2 in one pass (no tile round trip)
      fdm_pass_fused2<NA, NL, DIM, decltype(scale), NA, TAILK>(tile, trash, P, Q, scale, sBt[1], sBt[2]);
      P.template load_as<NL>(bwd[1]);
      __syncthreads();
    } else {
      fdm_pass<T, NA, NL, DIM, 2, decltype(scale), NA, TAILK>(tile, trash, P, scale, sBt[1]);
      __syncthreads();
      P.template load_as<NL>(bwd[1]);
      fdm_pass<T, NA, NL, DIM, 2, NoPost, NA, TAILK>(tile, trash, Q, NoPost(), sBt[2]);
      __syncthreads();
    }
    Q.template load_as<NA>(bwd[0]);
    fdm_pass<T, NA, NL, DIM, 1, NoPost, NA, TAILK>(tile, trash, P, NoPost(), sBt[3]);
    __syncthreads();
    fdm_pass<T, NA, NL, DIM, 0, NoPost, NA>(tile, trash, Q);
    __syncthreads();
  } else {
    fdm_pass_any<T, NA, NL, DIM, 0>(tile, trash, fwd[0], bwd[0]);
    __syncthreads();
    if constexpr (DIM == 3) {
      fdm_pass_any<T, NA, NL, DIM, 1>(tile, trash, fwd[1], bwd[1]);
      __syncthreads();
      fdm_pass_any<T, NA, NL, DIM, 2>(tile, trash, fwd[2], bwd[2], scale);
    } else {
      fdm_pass_any<T, NA, NL, DIM, 1>(tile, trash, fwd[1], bwd[1], scale);
    }
    __syncthreads();
    if constexpr (DIM == 3) {
      fdm_pass_any<T, NA, NL, DIM, 2>(tile, trash, bwd[2], fwd[2]);
      __syncthreads();
    }
    fdm_pass_any<T, NA, NL, DIM, 1>(tile, trash, bwd[1], fwd[1]);
    __syncthreads();
    fdm_pass_any<T, NA, NL, DIM, 0>(tile, trash, bwd[0], fwd[0]);
    __syncthreads();
  }
  // weighted result w_s (.) Delta u_s in grid-natural order; row weight w1 w2
  const auto row_w = [&](int rw) -> T {
    if constexpr (DIM == 3) return wv[1][rw % S::L1] * wv[2][rw / S::L1];
    else return wv[1][rw];
  };
  T* dst = out + (int64_t)pid * TS;
  if constexpr (G2D) {
    const int o0 = tid & 15, rstep = nth >> 4;
    if (o0 < S::L0) {
      const T w0 = wv[0][o0];
      const int pc = o0 * S::C0;
      for (int rw = tid >> 4; rw < S::NROW; rw += rstep) dst[rw * S::L0 + o0] = (w0 * row_w(rw)) * tile[rowpos[rw] + pc];
    }
  } else {
    for (int q = tid; q < TS; q += nth) {
      const int o0 = q % S::L0, rw = q / S::L0;
      dst[q] = (wv[0][o0] * row_w(rw)) * tile[rowpos[rw] + o0 * S::C0];
    }
  }
}

template <class T, int DIM, int NA, int NL, int ND, bool BATCH>
void fdm_launch_nd(const FdmArgs<T>& a, const BatchList<FdmArgs<T>>& bl, int nlog, int th, size_t shm,
                   hipStream_t s) {
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)fdm_kernel<T, DIM, NA, NL, ND, BATCH>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipLaunchKernelGGL((fdm_kernel<T, DIM, NA, NL, ND, BATCH>), dim3(xcd_grid(nlog)), dim3(th), shm, s, a, bl, nlog);
}

// waves: wavefronts per block (1 .. 8; 0 = default), the shape the autotuner picks.
template <class T, int DIM, int NA, int NL, bool BATCH>
int fdm_go(int nd, const FdmArgs<T>& a, const BatchList<FdmArgs<T>>& bl, int nlog, int waves, hipStream_t s) {
  constexpr size_t shm = fdm_shmem<T, NA, NL, DIM>();
  const int th = (waves >= 1 && waves <= 8) ? 64 * waves : fdm_threads<NA, NL, DIM>();
  if (nd < 0) {
    if constexpr (NA == NL) {
      fdm_launch_nd<T, DIM, NA, NL, -1, BATCH>(a, bl, nlog, th, shm, s);
      return 0;
    }
    return -4;
  }
  if (nd == 0) fdm_launch_nd<T, DIM, NA, NL, 0, BATCH>(a, bl, nlog, th, shm, s);
  else if (nd == 1) fdm_launch_nd<T, DIM, NA, NL, 1, BATCH>(a, bl, nlog, th, shm, s);
  else if constexpr (DIM == 3) fdm_launch_nd<T, DIM, NA, NL, 2, BATCH>(a, bl, nlog, th, shm, s);
  else return -4;
  return 0;
}

template <class T, int DIM, int NA, int NL>
int fdm_launch_t(const LevelDev<T>& L, int nd, const T* r, T* out, int npx, int npy, int npz,
                 int waves, const PatchLat& lat, hipStream_t s) {
  FdmArgs<T> a;
  a.L = L;
  a.r = r;
  a.out = out;
  a.npx = npx;
  a.npy = npy;
  a.npz = npz;
  a.lat = lat;
  const int npatch = npx * npy * (DIM == 3 ? npz : 1);
  return fdm_go<T, DIM, NA, NL, false>(nd, a, BatchList<FdmArgs<T>>{}, npatch, waves, s);
}

// One launch over the patch solves of many grids (same tile and normal): ntot
// logical blocks, one per patch, grid g's patches in the range of bl.
template <class T, int DIM, int NA, int NL>
int fdm_batch_launch(int nd, const BatchList<FdmArgs<T>>& bl, int ntot, int waves, hipStream_t s) {
  return fdm_go<T, DIM, NA, NL, true>(nd, FdmArgs<T>{}, bl, ntot, waves, s);
}

// ================================================================ multiplicative update
// u += R_s^T Delta u_s, unweighted, for the patches of one launch of the patch
// solve (a colour class: their node sets are disjoint, so every node receives
// at most one value and no two threads write the same entry).  One block per
// patch (its index among the launch's patches, as the patch solve numbered
// them), threads over its tile in grid-natural order; positions outside a
// Dirichlet domain are skipped.
template <class T, int DIM>
__global__ void __launch_bounds__(256) mult_update_kernel(LevelDev<T> L, int nd, int NA, int NL, PatchLat lat,
                                                          int npx, int npy, const T* __restrict__ buf,
                                                          T* __restrict__ u) {
  if (inactive(L.active)) return;
  const int pid = blockIdx.x;
  int p[3];
  p[0] = lat.start[0] + lat.stride[0] * (pid % npx);
  p[1] = lat.start[1] + lat.stride[1] * ((pid / npx) % npy);
  p[2] = DIM == 3 ? lat.start[2] + lat.stride[2] * (pid / (npx * npy)) : 0;
  const int* go[3] = {nullptr, nullptr, nullptr};
  int len[3] = {1, 1, 1};
  for (int d = 0; d < DIM; ++d) {
    const bool fc = d == nd;
    len[d] = fc ? NA : NL;
    go[d] = fc ? L.dir[d].goff_fc + p[d] * NA : L.dir[d].goff_ec + p[d] * NL;
  }
  const int ts = len[0] * len[1] * len[2];
  const T* src = buf + (int64_t)pid * ts;
  for (int q = threadIdx.x; q < ts; q += blockDim.x) {
    const int o0 = q % len[0], rw = q / len[0];
    const int o1 = rw % len[1], o2 = rw / len[1];
    const int g0 = go[0][o0], g1 = go[1][o1], g2 = DIM == 3 ? go[2][o2] : 0;
    if ((g0 | g1 | g2) < 0) continue;
    u[g0 + g1 + g2] += src[q];
  }
}

template <class T, int DIM>
int mult_update_launch(const LevelDev<T>& L, int nd, int NA, int NL, const PatchLat& lat, int npx, int npy,
                       int npz, const T* buf, T* u, hipStream_t s) {
  const int npatch = npx * npy * (DIM == 3 ? npz : 1);
  if (npatch <= 0) return 0;
  hipLaunchKernelGGL((mult_update_kernel<T, DIM>), dim3(npatch), dim3(256), 0, s, L, nd, NA, NL, lat, npx, npy, buf,
                     u);
  return 0;
}

// ================================================================ overlap summation
// u += sum_s R_s^T (w_s Delta u_s) (assign: u = the sum, for u = 0 on entry),
// gathered per node in a fixed order over the
// (at most 2 x 3 x 3) covering patches: deterministic, no atomics.  One block
// per group of elements; per element and direction the candidate patches of
// each local index are tabulated in LDS as address components, so a node's sum
// is a few loads at addresses Ax[i] + Ay[j] + Az[k].
template <int NP, int DIM>
constexpr int combine_epb() {
  return imax(1, 256 / ipow(NP, DIM));
}
// Large elements are split over several blocks of at most COMBINE_CHUNK nodes
// (a whole P = 32 element per block left 512 blocks, each thread looping 140
// times through latency-bound candidate loads).
constexpr int COMBINE_CHUNK = 2048;
template <int NP, int DIM>
constexpr int combine_bpe() {
  return combine_epb<NP, DIM>() == 1 ? (ipow(NP, DIM) + COMBINE_CHUNK - 1) / COMBINE_CHUNK : 1;
}

template <class T>
struct CombArgs {
  LevelDev<T> L;
  const T* buf = nullptr;  // the patch solve's weighted corrections
  T* u = nullptr;
  int nd = -1, NA = 0, NL = 0;
  int npx = 1, npy = 1, npz = 1;
  int nblk = 0;
  int assign = 0;
};

// BATCH: the arguments come from the work list bl (ntot logical blocks in all)
template <class T, int DIM, int NP, int MAXC, bool BATCH = false>
__global__ void __launch_bounds__(256) combine_kernel(CombArgs<T> a0, BatchList<CombArgs<T>> bl, int ntot) {
  constexpr int NE = ipow(NP, DIM), EPB = combine_epb<NP, DIM>(), BPE = combine_bpe<NP, DIM>();
  constexpr int P = NP - 1;
  constexpr int CZ = DIM == 3 ? MAXC : 1;
  __shared__ int64_t cadr[EPB][3][NP][MAXC];
  __shared__ int ccnt[EPB][3][NP];
  __shared__ __align__(16) int sargs_raw[BATCH ? sizeof(CombArgs<T>) / sizeof(int) : 1];
  CombArgs<T>* sargs = reinterpret_cast<CombArgs<T>*>(sargs_raw);
  const CombArgs<T>* ap;
  int blk;
  if constexpr (BATCH) {
    const int b = xcd_block(ntot);
    if (b < 0) return;
    blk = batch_pick(bl, b, sargs);
    ap = sargs;
  } else {
    blk = xcd_block(a0.nblk);
    if (blk < 0) return;
    ap = &a0;
  }
  const LevelDev<T>& L = ap->L;
  const T* __restrict__ buf = ap->buf;
  T* __restrict__ u = ap->u;
  const int nd = ap->nd, NA = ap->NA, NL = ap->NL, npx = ap->npx, npy = ap->npy;
  const bool assign = ap->assign != 0;
  if (inactive(L.active)) return;
  // BPE > 1: block blk takes nodes [q_lo, q_hi) of element blk / BPE
  const int e0 = BPE > 1 ? blk / BPE : blk * EPB;
  const int ne = BPE > 1 ? 1 : imin(EPB, L.n_elem - e0);
  const int q_lo = BPE > 1 ? (blk % BPE) * COMBINE_CHUNK : 0;
  const int q_hi = BPE > 1 ? imin(NE, q_lo + COMBINE_CHUNK) : ne * NE;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int N1 = L.dir[0].N, N2 = L.dir[1].N, NO = L.NO;
  int len[3] = {1, 1, 1};
  for (int d = 0; d < DIM; ++d) len[d] = (d == nd) ? NA : NL;
  const int64_t TS = (int64_t)len[0] * len[1] * len[2];
  const int64_t pst[3] = {1, npx, (int64_t)npx * npy};
  const int64_t ost[3] = {1, len[0], (int64_t)len[0] * len[1]};
  for (int q = tid; q < ne * DIM * NP; q += nth) {
    const int el = q / (DIM * NP), rem = q - el * DIM * NP, d = rem / NP, i = rem - d * NP;
    const int e = e0 + el;
    const int md = d == 0 ? e % N1 : (d == 1 ? (DIM == 3 ? (e / N1) % N2 : e / N1) : e / (N1 * N2));
    const DirDev<T>& dd = L.dir[d];
    const int N = dd.N;
    int c = 0;
    int cp[3], co[3];
    if (d == nd) {  // faces m (tile position P + i, needs i < P) and m + 1 (position i - 1, needs i >= 1)
      if (i < P) { cp[c] = md; co[c++] = P + i; }
      if (i >= 1) { cp[c] = dd.periodic ? (md + 1) % N : md + 1; co[c++] = i - 1; }
    } else {        // element-centred patches m - 1, m, m + 1
      if (i < NO && (dd.periodic || md > 0)) { cp[c] = (md - 1 + N) % N; co[c++] = NP + NO + i; }
      cp[c] = md; co[c++] = i + NO;
      if (i >= NP - NO && (dd.periodic || md < N - 1)) { cp[c] = (md + 1) % N; co[c++] = i - NP + NO; }
    }
    ccnt[el][d][i] = c;
    for (int k = 0; k < MAXC; ++k) cadr[el][d][i][k] = k < c ? cp[k] * pst[d] * TS + co[k] * ost[d] : 0;
  }
  if (DIM == 2)
    for (int q = tid; q < ne; q += nth) {
      ccnt[q][2][0] = 1;
      for (int k = 0; k < MAXC; ++k) cadr[q][2][0][k] = 0;
    }
  __syncthreads();
  // each node: all its (at most MAXC per direction) candidates are loaded before
  // the sum, then added in a fixed order (z, y, x candidates)
  const int64_t g0 = (int64_t)e0 * NE;
  for (int q = q_lo + tid; q < q_hi; q += nth) {
    const int el = q / NE, loc = q - el * NE;
    const int i = loc % NP, j = (loc / NP) % NP, k = DIM == 3 ? loc / (NP * NP) : 0;
    const int nx = ccnt[el][0][i], ny = ccnt[el][1][j], nz = ccnt[el][2][k];
    T v[CZ][MAXC][MAXC];
#pragma unroll
    for (int c = 0; c < CZ; ++c)
#pragma unroll
      for (int b = 0; b < MAXC; ++b)
#pragma unroll
        for (int a = 0; a < MAXC; ++a) {
          // invalid candidates are not loaded (their lanes are masked off: on
          // average about half of the 2 x 2 x 2 slots are empty) and add 0
          const bool ok = c < nz && b < ny && a < nx;
          T val = T(0);
          if (ok) val = buf[cadr[el][2][k][c] + cadr[el][1][j][b] + cadr[el][0][i][a]];
          v[c][b][a] = val;
        }
    T s = 0;
#pragma unroll
    for (int c = 0; c < CZ; ++c)
#pragma unroll
      for (int b = 0; b < MAXC; ++b)
#pragma unroll
        for (int a = 0; a < MAXC; ++a)
          s += T(c < nz && b < ny && a < nx ? 1 : 0) * v[c][b][a];  // s + 0 v = s: order unchanged
    if (assign)
      u[g0 + q] = s;
    else
      u[g0 + q] += s;
  }
}

// Blocks of one grid's overlap summation.
template <int DIM, int NP>
int combine_blocks(int n_elem) {
  constexpr int EPB = combine_epb<NP, DIM>(), BPE = combine_bpe<NP, DIM>();
  return BPE > 1 ? n_elem * BPE : (n_elem + EPB - 1) / EPB;
}
// Candidate slots per node and direction: three covering element-centred
// patches in one direction only when 2 N_O > N_P.
inline int combine_maxc(int NP, int NO) { return 2 * NO > NP ? 3 : 2; }

template <class T, int DIM, int NP>
int combine_launch_t(const LevelDev<T>& L, int nd, int NA, int NL, const T* buf, T* u, int npx,
                     int npy, int npz, bool assign, hipStream_t s) {
  CombArgs<T> a;
  a.L = L;
  a.buf = buf;
  a.u = u;
  a.nd = nd;
  a.NA = NA;
  a.NL = NL;
  a.npx = npx;
  a.npy = npy;
  a.npz = npz;
  a.nblk = combine_blocks<DIM, NP>(L.n_elem);
  a.assign = assign ? 1 : 0;
  if (combine_maxc(NP, L.NO) == 3)
    hipLaunchKernelGGL((combine_kernel<T, DIM, NP, 3, false>), dim3(xcd_grid(a.nblk)), dim3(256), 0, s, a,
                       BatchList<CombArgs<T>>{}, a.nblk);
  else
    hipLaunchKernelGGL((combine_kernel<T, DIM, NP, 2, false>), dim3(xcd_grid(a.nblk)), dim3(256), 0, s, a,
                       BatchList<CombArgs<T>>{}, a.nblk);
  return 0;
}

// One launch over the overlap summations of many grids (same NP and candidate
// slots maxc): ntot logical blocks, grid g's combine_blocks in the range of bl.
template <class T, int DIM, int NP>
int combine_batch_launch(int maxc, const BatchList<CombArgs<T>>& bl, int ntot, hipStream_t s) {
  if (maxc == 3)
    hipLaunchKernelGGL((combine_kernel<T, DIM, NP, 3, true>), dim3(xcd_grid(ntot)), dim3(256), 0, s, CombArgs<T>{},
                       bl, ntot);
  else
    hipLaunchKernelGGL((combine_kernel<T, DIM, NP, 2, true>), dim3(xcd_grid(ntot)), dim3(256), 0, s, CombArgs<T>{},
                       bl, ntot);
  return 0;
}

// ================================================================ p-transfers
// Element-local tensor-product contractions with the embedded interpolation J
// (NPf x NPc).  RESTRICT: out_c = (J^T x J^T x J^T) in_f.  Otherwise:
// out_f += (J x J x J) in_c.  One block per group of elements; LDS ping-pong.
constexpr int XFER_THREADS = 256;  // block size of transfer_kernel (its copies unroll over it)
template <int NPF, int DIM>
constexpr int xfer_epb() {
  return imax(1, 512 / ipow(NPF, DIM));
}

// One contraction pass of the transfer along direction D, all extents known at
// compile time: before the pass directions < D have NOUT points and the others
// NIN; the pass maps direction D from NIN to NOUT points.
template <class T, int DIM, int NIN, int NOUT, int NEF, int D, bool RESTRICT, int NPC>
__device__ __forceinline__ void xfer_pass(const T* __restrict__ sJ, const T* __restrict__ src,
                                          T* __restrict__ dst, int ne) {
  constexpr int n0 = D > 0 ? NOUT : NIN, n1 = D > 1 ? NOUT : NIN;
  constexpr int m0 = NOUT * (D == 0) + n0 * (D != 0);
  constexpr int m1 = DIM >= 2 ? (D >= 1 ? NOUT : NIN) : 1;
  constexpr int m2 = DIM == 3 ? (D == 2 ? NOUT : NIN) : 1;
  constexpr int per = m0 * m1 * m2;
  constexpr int SK = D == 0 ? 1 : (D == 1 ? n0 : n0 * n1);  // source stride of direction D
  for (int q = threadIdx.x; q < ne * per; q += blockDim.x) {
    const int el = q / per, r = q - el * per;
    const int i0 = r % m0, i1 = (r / m0) % m1, i2 = r / (m0 * m1);
    const int iout = D == 0 ? i0 : (D == 1 ? i1 : i2);
    // source position with the direction-D index set to 0
    const int j0 = D == 0 ? 0 : i0, j1 = D == 1 ? 0 : i1, j2 = D == 2 ? 0 : i2;
    const T* sp = src + el * NEF + (j2 * n1 + j1) * n0 + j0;
    T s = 0;
#pragma unroll
    for (int k = 0; k < NIN; ++k) {
      const T jv = RESTRICT ? sJ[k * NPC + iout] : sJ[iout * NPC + k];
      s += jv * sp[k * SK];
    }
    dst[el * NEF + r] = s;
  }
}

template <class T>
struct XferArgs {
  const T* J = nullptr;
  int n_elem = 0;
  const T* in = nullptr;
  T* out = nullptr;
  const int* active = nullptr;
};

// BATCH: the arguments come from the work list bl (ntot logical blocks in all)
template <class T, int DIM, int NPF, int NPC, bool RESTRICT, bool BATCH = false>
__global__ void __launch_bounds__(512) transfer_kernel(XferArgs<T> a0, BatchList<XferArgs<T>> bl, int ntot) {
  __shared__ __align__(16) int sargs_raw[BATCH ? sizeof(XferArgs<T>) / sizeof(int) : 1];
  XferArgs<T>* sargs = reinterpret_cast<XferArgs<T>*>(sargs_raw);
  const XferArgs<T>* ap;
  int blk = blockIdx.x;
  if constexpr (BATCH) {
    const int b = xcd_block(ntot);
    if (b < 0) return;
    blk = batch_pick(bl, b, sargs);
    ap = sargs;
  } else {
    ap = &a0;
  }
  const T* __restrict__ J = ap->J;
  const int n_elem = ap->n_elem;
  const T* __restrict__ in = ap->in;
  T* __restrict__ out = ap->out;
  if (inactive(ap->active)) return;
  constexpr int NEF = ipow(NPF, DIM), EPB = xfer_epb<NPF, DIM>();
  constexpr int NIN = RESTRICT ? NPF : NPC, NOUT = RESTRICT ? NPC : NPF;
  constexpr int NEI = ipow(NIN, DIM), NEO = ipow(NOUT, DIM);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* bufA = reinterpret_cast<T*>(smem_raw);
  T* bufB = bufA + EPB * NEF;
  __shared__ T sJ[NPF * NPC];
  const int e0 = blk * EPB;
  const int ne = imin(EPB, n_elem - e0);
  staged_copy<T, XFER_THREADS, NPF * NPC>([&](int q) { return J[q]; }, [&](int q, T v) { sJ[q] = v; });
  staged_copy<T, XFER_THREADS, EPB * NEI>([&](int q) { return in[(int64_t)e0 * NEI + q]; },
                                          [&](int q, T v) {
                                            const int el = q / NEI;
                                            bufA[el * NEF + q - el * NEI] = v;  // per-element stride NEF in LDS
                                          },
                                          ne * NEI);
  __syncthreads();
  xfer_pass<T, DIM, NIN, NOUT, NEF, 0, RESTRICT, NPC>(sJ, bufA, bufB, ne);
  __syncthreads();
  xfer_pass<T, DIM, NIN, NOUT, NEF, 1, RESTRICT, NPC>(sJ, bufB, bufA, ne);
  __syncthreads();
  const T* res = bufA;
  if constexpr (DIM == 3) {
    xfer_pass<T, DIM, NIN, NOUT, NEF, 2, RESTRICT, NPC>(sJ, bufA, bufB, ne);
    __syncthreads();
    res = bufB;
  }
  const auto rv = [&](int q) {
    const int el = q / NEO;
    return res[el * NEF + q - el * NEO];
  };
  T* o = out + (int64_t)e0 * NEO;
  if constexpr (RESTRICT)
    staged_copy<T, XFER_THREADS, EPB * NEO>(rv, [&](int q, T v) { o[q] = v; }, ne * NEO);
  else
    staged_copy<T, XFER_THREADS, EPB * NEO>([&](int q) { return o[q]; }, [&](int q, T v) { o[q] = v + rv(q); },
                                            ne * NEO);
}

// Blocks of one grid's transfer.
template <int DIM, int NPF>
int xfer_blocks(int n_elem) {
  constexpr int EPB = xfer_epb<NPF, DIM>();
  return (n_elem + EPB - 1) / EPB;
}

template <class T, int DIM, int NPF, int NPC, bool RESTRICT, bool BATCH>
void transfer_go(const XferArgs<T>& a, const BatchList<XferArgs<T>>& bl, int nblk, hipStream_t s) {
  constexpr int EPB = xfer_epb<NPF, DIM>();
  const size_t shm = 2 * (size_t)EPB * ipow(NPF, DIM) * sizeof(T);
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)transfer_kernel<T, DIM, NPF, NPC, RESTRICT, BATCH>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  const int grid = BATCH ? xcd_grid(nblk) : nblk;
  hipLaunchKernelGGL((transfer_kernel<T, DIM, NPF, NPC, RESTRICT, BATCH>), dim3(grid), dim3(XFER_THREADS), shm, s,
                     a, bl, nblk);
}

template <class T, int DIM, int NPF, int NPC, bool RESTRICT>
int transfer_launch_t(const T* J, int n_elem, const T* in, T* out, const int* active, hipStream_t s) {
  XferArgs<T> a;
  a.J = J;
  a.n_elem = n_elem;
  a.in = in;
  a.out = out;
  a.active = active;
  transfer_go<T, DIM, NPF, NPC, RESTRICT, false>(a, BatchList<XferArgs<T>>{}, xfer_blocks<DIM, NPF>(n_elem), s);
  return 0;
}

// One launch over the transfers of many grids (same order pair and direction):
// ntot logical blocks, grid g's xfer_blocks in the range of bl.
template <class T, int DIM, int NPF, int NPC>
int transfer_batch_launch(bool restrict_, const BatchList<XferArgs<T>>& bl, int ntot, hipStream_t s) {
  if (restrict_) transfer_go<T, DIM, NPF, NPC, true, true>(XferArgs<T>{}, bl, ntot, s);
  else transfer_go<T, DIM, NPF, NPC, false, true>(XferArgs<T>{}, bl, ntot, s);
  return 0;
}

// ================================================================ dispatch (instantiated per T, DIM)
template <class T, int DIM>
struct Kern {
  // scratch: apply_big_scratch(n_elem, NP) elements (3D levels with NP = 33 only).
  // mode 3 (residual restricted to the coarser level, y coarse) returns -4 where
  // it is not built (large elements): the caller then runs mode 1 and transfer.
  static int apply(const LevelDev<T>& L, int mode, const T* x, const T* f, T* y, T* scratch, double* part,
                   int* nblk, hipStream_t s);
  // lat: the patches of this launch (all of them: PatchLat{}); large tiles
  // (3D P = 32) take only the whole partition
  static int fdm(const LevelDev<T>& L, int nd, int NA, int NL, const T* r, T* out, int npx, int npy,
                 int npz, int waves, const PatchLat& lat, hipStream_t s);
  // u += the unweighted corrections of one patch-solve launch (disjoint patches)
  static int mult_update(const LevelDev<T>& L, int nd, int NA, int NL, const PatchLat& lat, int npx, int npy,
                         int npz, const T* buf, T* u, hipStream_t s);
  // Batched launches (work lists over many grids, see BatchList): the same
  // kernels as above with per-grid arguments.  Block counts per grid:
  // apply_blocks, one per patch, combine_blocks, xfer_blocks.  -4 where the
  // template is not built.
  static int apply_blocks_of(int NP, int n_elem);
  static int combine_blocks_of(int NP, int n_elem);
  static int xfer_blocks_of(int NPF, int n_elem);
  static bool mode3_ok(const LevelDev<T>& L);
  static int apply_batch(int NP, int mode, const BatchList<ApplyArgs<T>>& bl, int ntot, hipStream_t s);
  static int fdm_batch(int nd, int NA, int NL, const BatchList<FdmArgs<T>>& bl, int ntot, int waves, hipStream_t s);
  static int combine_batch(int NP, int maxc, const BatchList<CombArgs<T>>& bl, int ntot, hipStream_t s);
  static int transfer_batch(int NPF, int NPC, bool restrict_, const BatchList<XferArgs<T>>& bl, int ntot,
                            hipStream_t s);
  static bool fdm_supported(int NA, int NL);
  // the order has compiled kernels (others run the run-time forms of kernels_gen.hpp)
  static bool order_compiled(int NP);
  // the tile's solve runs in LDS (not the large-tile stages through global memory)
  static bool fdm_in_lds(int NA, int NL);
  // assign: u = the overlap sum (u is zero on entry) instead of u += it
  static int combine(const LevelDev<T>& L, int nd, int NA, int NL, const T* buf, T* u, int npx,
                     int npy, int npz, bool assign, hipStream_t s);
  // tmp: scratch of transfer_big_scratch(n_elem, NP, NPc) elements (3D levels with NP = 33 only)
  static int transfer(const LevelDev<T>& Lf, bool restrict_, const T* in, T* out, T* tmp, hipStream_t s);
  // Continuous spectral-element levels (lattice vectors, kernels_se.hpp).
  // ebuf: element-major scratch of n_elem * NP^DIM elements.  Modes 0 and 1.
  static int se_apply(const LevelDev<T>& L, int mode, const T* x, const T* f, T* y, T* ebuf, hipStream_t s);
  static int se_combine(const LevelDev<T>& L, int NA, const T* buf, T* u, bool assign, hipStream_t s);
  // ebuf (restriction only): n_elem * NPc^DIM elements
  static int se_transfer(const LevelDev<T>& Lf, const LevelDev<T>& Lc, bool restrict_, const T* in, T* out,
                         T* ebuf, hipStream_t s);
};

}  // namespace dgmg

// Runtime -> template dispatch for the kernels of kernels.hpp.  Included by one
// translation unit per (precision, dimension) so they compile in parallel.
#pragma once

#include "kernels.hpp"
#include "kernels_big.hpp"
#include "kernels_se.hpp"
#include "kernels_gen.hpp"

namespace dgmg {

// Orders with kernels: P in {1, 2, 3, 4, 6, 8, 12, 16, 32}  (NP = P + 1).
#define DGMG_NP_LIST(X) X(2) X(3) X(4) X(5) X(7) X(9) X(13) X(17) X(33)
// Transfer pairs (NP fine, NP coarse) for P -> floor(P / 2).
#define DGMG_XFER_LIST(X) X(3, 2) X(4, 2) X(5, 3) X(7, 4) X(9, 5) X(13, 7) X(17, 9) X(33, 17)
// 3D elements with NP = BIG_NP and patch tiles beyond LDS use kernels_big.hpp.
constexpr size_t LDS_BYTES = 160 * 1024;  // gfx950 LDS per workgroup
// Patch tiles (NA, NL): element-centred (n, n) with n = NP + 2 N_O and
// face-centred (2P, NP + 2 N_O) for the overlaps N_O the level rules produce
// (and N_O = 0, 1 for the zero-overlap variants).
#define DGMG_FDM_LIST(X)                                                                    \
  X(3, 3) X(4, 4) X(5, 5) X(6, 6) X(7, 7) X(9, 9) X(11, 11) X(13, 13) X(15, 15) X(17, 17) \
  X(19, 19) X(21, 21) X(23, 23) X(4, 3) X(4, 5) X(6, 4) X(8, 5) X(8, 7) X(8, 9) X(12, 7)  \
  X(12, 9) X(12, 11) X(16, 9) X(16, 11) X(16, 13) X(16, 15) X(24, 13) X(24, 17) X(24, 19) \
  X(32, 17) X(32, 21) X(32, 23) X(33, 33) X(35, 35) X(43, 43) X(64, 33) X(64, 35) X(64, 43)
// Tiles built for 2D only: the continuous element-centred patches of P_l = 32.
#define DGMG_FDM_LIST_2D(X) X(41, 41)

template <class T, int DIM>
int Kern<T, DIM>::apply(const LevelDev<T>& L, int mode, const T* x, const T* f, T* y, T* scratch, double* part,
                        int* nblk, hipStream_t s) {
  switch (L.NP) {
#define DGMG_CASE(NP)                                                              \
  case NP:                                                                         \
    if constexpr (DIM == 3 && NP == BIG_NP)                                        \
      return mode == 3 ? -4 : apply_big_launch<T, NP>(L, mode, x, f, y, scratch, part, nblk, s); \
    else                                                                           \
      return apply_launch<T, DIM, NP>(L, mode, x, f, y, part, nblk, s);
    DGMG_NP_LIST(DGMG_CASE)
#undef DGMG_CASE
    default:  // orders without compiled kernels: the run-time form (modes 0 and 1)
      return gen_apply_launch<T>(L, mode, x, f, y, s);
  }
}

template <class T, int DIM>
bool Kern<T, DIM>::order_compiled(int NP) {
  switch (NP) {
#define DGMG_CASE(N) \
  case N: return true;
    DGMG_NP_LIST(DGMG_CASE)
#undef DGMG_CASE
    default: return false;
  }
}

template <class T, int DIM>
bool Kern<T, DIM>::fdm_supported(int NA, int NL) {
#define DGMG_CASE(A, B) \
  if (NA == A && NL == B) return true;
  DGMG_FDM_LIST(DGMG_CASE)
  if constexpr (DIM == 2) {
    DGMG_FDM_LIST_2D(DGMG_CASE)
  }
#undef DGMG_CASE
  return gen_fdm_fits<T>(DIM, NA, NL);  // the run-time tile form
}

template <class T, int DIM>
bool Kern<T, DIM>::fdm_in_lds(int NA, int NL) {
#define DGMG_CASE(A, B) \
  if (NA == A && NL == B) return !(DIM == 3 && fdm_lds_total<T, A, B, DIM>() > LDS_BYTES);
  DGMG_FDM_LIST(DGMG_CASE)
  if constexpr (DIM == 2) {
    DGMG_FDM_LIST_2D(DGMG_CASE)
  }
#undef DGMG_CASE
  return gen_fdm_fits<T>(DIM, NA, NL);
}

template <class T, int DIM>
int Kern<T, DIM>::fdm(const LevelDev<T>& L, int nd, int NA, int NL, const T* r, T* out, int npx,
                      int npy, int npz, int waves, const PatchLat& lat, hipStream_t s) {
  const bool whole = lat.start[0] == 0 && lat.start[1] == 0 && lat.start[2] == 0 && lat.stride[0] == 1 &&
                     lat.stride[1] == 1 && lat.stride[2] == 1;
#define DGMG_CASE(A, B)                                                                   \
  if (NA == A && NL == B) {                                                               \
    if constexpr (DIM == 3 && fdm_lds_total<T, A, B, DIM>() > LDS_BYTES)                  \
      return whole ? fdm_big_launch<T, A, B>(L, nd, r, out, npx, npy, npz, s) : -4;       \
    else                                                                                  \
      return fdm_launch_t<T, DIM, A, B>(L, nd, r, out, npx, npy, npz, waves, lat, s);     \
  }
  DGMG_FDM_LIST(DGMG_CASE)
#undef DGMG_CASE
  if constexpr (DIM == 2) {
#define DGMG_CASE(A, B) \
  if (NA == A && NL == B) return fdm_launch_t<T, DIM, A, B>(L, nd, r, out, npx, npy, npz, waves, lat, s);
    DGMG_FDM_LIST_2D(DGMG_CASE)
#undef DGMG_CASE
  }
  return gen_fdm_launch<T>(L, nd, NA, NL, r, out, npx, npy, npz, lat, s);  // run-time tile
}

template <class T, int DIM>
int Kern<T, DIM>::mult_update(const LevelDev<T>& L, int nd, int NA, int NL, const PatchLat& lat, int npx,
                              int npy, int npz, const T* buf, T* u, hipStream_t s) {
  return mult_update_launch<T, DIM>(L, nd, NA, NL, lat, npx, npy, npz, buf, u, s);
}

template <class T, int DIM>
int Kern<T, DIM>::apply_blocks_of(int NP, int n_elem) {
  switch (NP) {
#define DGMG_CASE(N) \
  case N: return (DIM == 3 && N == BIG_NP) ? -4 : apply_blocks<DIM, N>(n_elem);
    DGMG_NP_LIST(DGMG_CASE)
#undef DGMG_CASE
    default: return -4;
  }
}

template <class T, int DIM>
int Kern<T, DIM>::combine_blocks_of(int NP, int n_elem) {
  switch (NP) {
#define DGMG_CASE(N) \
  case N: return combine_blocks<DIM, N>(n_elem);
    DGMG_NP_LIST(DGMG_CASE)
#undef DGMG_CASE
    default: return -4;
  }
}

template <class T, int DIM>
int Kern<T, DIM>::xfer_blocks_of(int NPF, int n_elem) {
  switch (NPF) {
#define DGMG_CASE(N) \
  case N: return (DIM == 3 && N == BIG_NP) ? -4 : xfer_blocks<DIM, N>(n_elem);
    DGMG_NP_LIST(DGMG_CASE)
#undef DGMG_CASE
    default: return -4;
  }
}

template <class T, int DIM>
bool Kern<T, DIM>::mode3_ok(const LevelDev<T>& L) {
  switch (L.NP) {
#define DGMG_CASE(N) \
  case N: return apply_mode3_ok<T, DIM, N>(L);
    DGMG_NP_LIST(DGMG_CASE)
#undef DGMG_CASE
    default: return false;
  }
}

template <class T, int DIM>
int Kern<T, DIM>::apply_batch(int NP, int mode, const BatchList<ApplyArgs<T>>& bl, int ntot, hipStream_t s) {
  switch (NP) {
#define DGMG_CASE(N)                                                   \
  case N:                                                              \
    if constexpr (DIM == 3 && N == BIG_NP)                             \
      return -4;                                                       \
    else                                                               \
      return apply_batch_launch<T, DIM, N>(mode, bl, ntot, s);
    DGMG_NP_LIST(DGMG_CASE)
#undef DGMG_CASE
    default: return -4;
  }
}

template <class T, int DIM>
int Kern<T, DIM>::fdm_batch(int nd, int NA, int NL, const BatchList<FdmArgs<T>>& bl, int ntot, int waves,
                            hipStream_t s) {
#define DGMG_CASE(A, B)                                                          \
  if (NA == A && NL == B) {                                                      \
    if constexpr (DIM == 3 && fdm_lds_total<T, A, B, DIM>() > LDS_BYTES)         \
      return -4;                                                                 \
    else                                                                         \
      return fdm_batch_launch<T, DIM, A, B>(nd, bl, ntot, waves, s);             \
  }
  DGMG_FDM_LIST(DGMG_CASE)
#undef DGMG_CASE
  return -4;
}

template <class T, int DIM>
int Kern<T, DIM>::combine_batch(int NP, int maxc, const BatchList<CombArgs<T>>& bl, int ntot, hipStream_t s) {
  switch (NP) {
#define DGMG_CASE(N) \
  case N: return combine_batch_launch<T, DIM, N>(maxc, bl, ntot, s);
    DGMG_NP_LIST(DGMG_CASE)
#undef DGMG_CASE
    default: return -4;
  }
}

template <class T, int DIM>
int Kern<T, DIM>::transfer_batch(int NPF, int NPC, bool restrict_, const BatchList<XferArgs<T>>& bl, int ntot,
                                 hipStream_t s) {
#define DGMG_CASE(F, C)                                                        \
  if (NPF == F && NPC == C) {                                                  \
    if constexpr (DIM == 3 && F == BIG_NP)                                     \
      return -4;                                                               \
    else                                                                       \
      return transfer_batch_launch<T, DIM, F, C>(restrict_, bl, ntot, s);      \
  }
  DGMG_XFER_LIST(DGMG_CASE)
#undef DGMG_CASE
  return -4;
}

template <class T, int DIM>
int Kern<T, DIM>::combine(const LevelDev<T>& L, int nd, int NA, int NL, const T* buf, T* u, int npx,
                          int npy, int npz, bool assign, hipStream_t s) {
  switch (L.NP) {
#define DGMG_CASE(NP) \
  case NP: return combine_launch_t<T, DIM, NP>(L, nd, NA, NL, buf, u, npx, npy, npz, assign, s);
    DGMG_NP_LIST(DGMG_CASE)
#undef DGMG_CASE
    default: return gen_combine_launch<T>(L, nd, NA, NL, buf, u, npx, npy, assign, s);
  }
}

template <class T, int DIM>
int Kern<T, DIM>::transfer(const LevelDev<T>& Lf, bool restrict_, const T* in, T* out, T* tmp,
                           hipStream_t s) {
#define DGMG_CASE(F, C)                                                                                \
  if (Lf.NP == F && Lf.NPc == C) {                                                                     \
    if constexpr (DIM == 3 && F == BIG_NP)                                                             \
      return transfer_big_launch<T, F, C>(Lf.J, Lf.n_elem, restrict_, in, out, tmp, Lf.active, s);    \
    else                                                                                               \
      return restrict_ ? transfer_launch_t<T, DIM, F, C, true>(Lf.J, Lf.n_elem, in, out, Lf.active, s) \
                       : transfer_launch_t<T, DIM, F, C, false>(Lf.J, Lf.n_elem, in, out, Lf.active, s); \
  }
  DGMG_XFER_LIST(DGMG_CASE)
#undef DGMG_CASE
  return gen_transfer_launch<T>(Lf, restrict_, in, out, s);  // run-time orders
}

template <class T, int DIM>
int Kern<T, DIM>::se_apply(const LevelDev<T>& L, int mode, const T* x, const T* f, T* y, T* ebuf, hipStream_t s) {
  switch (L.NP) {
#define DGMG_CASE(NP) \
  case NP: return se_apply_launch<T, DIM, NP>(L, mode, x, f, y, ebuf, s);
    DGMG_NP_LIST(DGMG_CASE)
#undef DGMG_CASE
    default: return -4;
  }
}

template <class T, int DIM>
int Kern<T, DIM>::se_combine(const LevelDev<T>& L, int NA, const T* buf, T* u, bool assign, hipStream_t s) {
  return se_combine_launch<T, DIM>(L, NA, buf, u, assign, s);
}

template <class T, int DIM>
int Kern<T, DIM>::se_transfer(const LevelDev<T>& Lf, const LevelDev<T>& Lc, bool restrict_, const T* in, T* out,
                              T* ebuf, hipStream_t s) {
#define DGMG_CASE(F, C) \
  if (Lf.NP == F && Lf.NPc == C) return se_transfer_launch<T, DIM, F, C>(Lf, Lc, restrict_, in, out, ebuf, s);
  DGMG_XFER_LIST(DGMG_CASE)
#undef DGMG_CASE
  return -4;
}

}  // namespace dgmg

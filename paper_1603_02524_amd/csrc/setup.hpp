// Host-side (FP64) construction of every table the device path needs.
//
// Sec. 2.4: GLL points and weights, differentiation and stiffness matrices,
// the global 1D operators of eq. (L:generic) (blocks from eq. (primal form)),
// Sec. 3.1: per-subdomain generalised eigenpairs and 1D weights,
// Sec. 3.2: level series and embedded interpolation.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace dgmg {

// 1D element coefficients used by the operator kernels, per element m:
enum ECoef {
  EC_TWO_DX = 0,  // 2 / dx_m
  EC_HALF_DX,     // dx_m / 2 (1D mass = HALF_DX * rho_i)
  EC_CL,          // lift/consistency factor of the left face: (1-2b)/dx_m, or 2/dx_m on a Dirichlet face
  EC_CNL,         // neighbour-derivative factor at the left face: (1+2b)/dx_{m-1}, 0 on a Dirichlet face
  EC_BL,          // penalty bracket B_{m-1/2} (mu_b on a Dirichlet face)
  EC_CR,          // (1+2b)/dx_m, or 2/dx_m on a Dirichlet face
  EC_CNR,         // (1-2b)/dx_{m+1}, 0 on a Dirichlet face
  EC_BR,          // B_{m+1/2} (mu_b on a Dirichlet face)
  EC_COUNT
};

struct Dir1D {
  int N = 0;
  bool periodic = false;
  int nl = 0;  // continuous levels: stored lattice nodes (N P - 1 Dirichlet, N P periodic)
  std::vector<double> dx;
  std::vector<double> ecoef;  // N * EC_COUNT
  std::vector<int> nbr;       // N * 2: left / right neighbour element, -1 at a Dirichlet face
  // element-centred patches (one per element), tile size n_ec = NP + 2 NO
  int n_ec = 0;
  std::vector<double> S_ec, lam_ec, w_ec;  // N * n*n (row-major S[k*n+j]), N*n, N*n
  // face-centred patches (normal direction), tile size n_fc = 2P
  int nf = 0, n_fc = 0;
  std::vector<double> S_fc, lam_fc, w_fc;
  // global generalised eigenpairs of (L_d, M_d) (coarsest level only), size G = N*NP
  int G = 0;
  std::vector<double> S_glob, lam_glob;  // G*G row-major, G
  int null_mode = -1;                    // index of the zero eigenvalue (periodic), else -1
};

struct LevelHost {
  int P = 1, NP = 2, NO = 0, dim = 3;
  bool se = false;  // continuous spectral-element level
  int64_t n_elem = 0, n_dof = 0;
  std::vector<double> rho, Ls, D;  // NP, NP*NP (row-major), NP*NP (D[i*NP+k] = phi_k'(eta_i))
  std::vector<double> J;           // NP x NPc interpolation from the next coarser level (row-major)
  int NPc = 0;
  Dir1D dir[3];
};

struct SetupParams {
  int dim = 3;
  int n[3] = {1, 1, 1};
  std::vector<double> dx[3];
  bool periodic[3] = {false, false, false};
  int P = 4;
  int flux = 0;
  double beta[3] = {0, 0, 0};
  double mu_star = 1.0;
  int smoother = 1;
  int overlap = -1;
  int weighting = 0;
  int disc = 0;  // 0: DG; 1: the continuous spectral-element counterpart (element-centred smoother only)
};

// Builds all levels (index 0 = coarsest, P = 1).  Returns an empty string on
// success, else an error message.
std::string build_levels(const SetupParams& sp, std::vector<LevelHost>& levels);

// Primitives (exposed for the host self-checks).
void gll_points(int P, std::vector<double>& eta, std::vector<double>& rho);
void gll_diff(int P, const std::vector<double>& eta, std::vector<double>& D);
int overlap_rule(int P_l, int overlap);
// Learned-weight variant of the face-centred smoother (not in the paper).
// Faces are enumerated level by level (l = 1 .. L), then by normal direction d,
// then by face index f = 0 .. nf_d - 1.
constexpr int FACE_FEATURES = 6;
int face_count(const std::vector<LevelHost>& levels);
// Features per face, FACE_FEATURES each: P_l / 32, log2(dx_left / h_lat) / 5,
// log2(dx_right / h_lat) / 5, 1 on a Dirichlet boundary face else 0, dim - 2,
// N_O,l / (P_l + 1).  h_lat is the geometric mean of the element sizes of the
// other directions; a missing neighbour element at a boundary face is replaced
// by the existing one.
void face_features(const std::vector<LevelHost>& levels, std::vector<double>& X);
// Normal weights of the face-centred patches of direction d on one level with a
// transition width theta_f and a damping omega_f per face:
//   w_f = omega_f * wt_f / (sum of wt_f' over the faces whose patch covers the node),
//   wt_f = 1/2 [1 + phi((1 - |xi_F|) / theta_f)]   (theta = 1: the weight of Sec. 3.1).
// Layout as Dir1D::w_fc (nf * n_fc, padding positions 0).
void fc_weights_param(const LevelHost& lv, int d, int kind, const double* theta, const double* omega,
                      std::vector<double>& w);

// Symmetric eigen-decomposition by the cyclic Jacobi method: A (n*n, row-major,
// destroyed) -> eigenvalues lam, eigenvectors as columns of V (row-major).
void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& lam, std::vector<double>& V);

}  // namespace dgmg

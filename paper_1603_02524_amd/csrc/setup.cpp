// Host-side FP64 setup: 1D spectral toolkit, DG operator coefficients,
// Schwarz patch eigenpairs and weights, level series and interpolation.
#include "setup.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <sstream>

namespace dgmg {

namespace {

// Legendre polynomial L_P(x) and L_{P-1}(x) by the three-term recurrence.
void legendre_pair(int P, double x, double& lp, double& lpm1) {
  double l0 = 1.0, l1 = x;
  if (P == 0) { lp = 1.0; lpm1 = 0.0; return; }
  for (int k = 1; k < P; ++k) {
    double l2 = ((2.0 * k + 1.0) * x * l1 - k * l0) / (k + 1.0);
    l0 = l1;
    l1 = l2;
  }
  lp = l1;
  lpm1 = l0;
}

double phi_tilde(double x, int kind) {
  switch (kind) {
    case 0: return (15.0 * x - 10.0 * x * x * x + 3.0 * x * x * x * x * x) / 8.0;  // quintic
    case 1: return (3.0 * x - x * x * x) / 2.0;                                       // cubic
    default: return 0.0;                                                             // arithmetic
  }
}

// Smoothed sign function phi of Sec. 3.1 (phi = 1 for the unweighted variant).
double phi(double x, int kind) {
  if (kind == 3) return 1.0;
  if (std::fabs(x) < 1.0) return phi_tilde(x, kind);
  return x > 0 ? 1.0 : (x < 0 ? -1.0 : 0.0);
}

// Generalised symmetric eigenproblem L S = M S Lambda with M diagonal > 0,
// S^T M S = I.  L: n*n row-major.
void gen_eigen(int n, const std::vector<double>& L, const std::vector<double>& m,
               std::vector<double>& S, std::vector<double>& lam) {
  std::vector<double> C(n * n), V;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      C[i * n + j] = 0.5 * (L[i * n + j] + L[j * n + i]) / std::sqrt(m[i] * m[j]);
  jacobi_eigen(n, C, lam, V);
  S.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) S[i * n + j] = V[i * n + j] / std::sqrt(m[i]);
}

}  // namespace

void gll_points(int P, std::vector<double>& eta, std::vector<double>& rho) {
  // Nodes: -1, 1 and the zeros of L_P'.  Newton iteration on L_P' with
  // L_P'' from the Legendre equation, started at Chebyshev-Lobatto points.
  eta.assign(P + 1, 0.0);
  rho.assign(P + 1, 0.0);
  eta[0] = -1.0;
  eta[P] = 1.0;
  for (int i = 1; i < P; ++i) {
    double x = -std::cos(M_PI * i / P);
    for (int it = 0; it < 100; ++it) {
      double lp, lpm1;
      legendre_pair(P, x, lp, lpm1);
      double d1 = P * (x * lp - lpm1) / (x * x - 1.0);           // L_P'
      double d2 = (2.0 * x * d1 - P * (P + 1.0) * lp) / (1.0 - x * x);  // L_P''
      double dx = d1 / d2;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    eta[i] = x;
  }
  std::sort(eta.begin(), eta.end());
  // symmetrise against round-off
  for (int i = 0; i <= P / 2; ++i) {
    double a = 0.5 * (eta[P - i] - eta[i]);
    eta[i] = -a;
    eta[P - i] = a;
  }
  if (P % 2 == 0) eta[P / 2] = 0.0;
  for (int i = 0; i <= P; ++i) {
    double lp, lpm1;
    legendre_pair(P, eta[i], lp, lpm1);
    rho[i] = 2.0 / (P * (P + 1.0) * lp * lp);
  }
}

void gll_diff(int P, const std::vector<double>& eta, std::vector<double>& D) {
  // Closed form of the GLL differentiation matrix:
  // D_ik = L_P(eta_i) / (L_P(eta_k) (eta_i - eta_k)), i != k;
  // D_00 = -P(P+1)/4, D_PP = P(P+1)/4, other diagonal entries 0.
  int NP = P + 1;
  std::vector<double> lp(NP);
  for (int i = 0; i < NP; ++i) {
    double a, b;
    legendre_pair(P, eta[i], a, b);
    lp[i] = a;
  }
  D.assign(NP * NP, 0.0);
  for (int i = 0; i < NP; ++i)
    for (int k = 0; k < NP; ++k)
      if (i != k) D[i * NP + k] = lp[i] / (lp[k] * (eta[i] - eta[k]));
  D[0] = -P * (P + 1.0) / 4.0;
  D[P * NP + P] = P * (P + 1.0) / 4.0;
}

int overlap_rule(int P_l, int overlap) {
  if (overlap == -1) return 1 + (P_l + 4) / 8;  // 1 + round(P_l / 8), halves up
  if (overlap == -2) return 1 + P_l / 8;        // 1 + floor(P_l / 8)
  return overlap;
}

void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& lam, std::vector<double>& V) {
  V.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  double norm = 0.0;
  for (int i = 0; i < n * n; ++i) norm += A[i] * A[i];
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    if (off <= 1e-34 * norm) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        // rotation in the (p, q) plane that annihilates A_pq
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        A[p * n + q] = 0.0;
        A[q * n + p] = 0.0;
        for (int k = 0; k < n; ++k) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
    }
  }
  lam.resize(n);
  for (int i = 0; i < n; ++i) lam[i] = A[i * n + i];
}

namespace {

// Element coefficients of eq. (L:generic) for direction data d at order P.
void element_coefficients(int P, const std::vector<double>& rho, double beta, double mu_star,
                          Dir1D& d) {
  const int N = d.N;
  d.ecoef.assign(N * EC_COUNT, 0.0);
  d.nbr.assign(N * 2, -1);
  const double rP = rho[P], r0 = rho[0];
  auto bracket = [&](double hl, double hr) {  // B at a face between elements of size hl | hr
    double mu0 = 1.0 / (2.0 * hl * rP) + 1.0 / (2.0 * hr * r0);
    double mu = (1.0 + mu_star) * mu0;
    return 2.0 * (beta * beta + beta) / (hl * rP) + 2.0 * (beta * beta - beta) / (hr * r0) + mu;
  };
  for (int m = 0; m < N; ++m) {
    double h = d.dx[m];
    double* c = &d.ecoef[m * EC_COUNT];
    c[EC_TWO_DX] = 2.0 / h;
    c[EC_HALF_DX] = 0.5 * h;
    bool hasl = d.periodic || m > 0, hasr = d.periodic || m < N - 1;
    int ml = (m - 1 + N) % N, mr = (m + 1) % N;
    if (hasl) {
      d.nbr[2 * m] = ml;
      c[EC_CL] = (1.0 - 2.0 * beta) / h;
      c[EC_CNL] = (1.0 + 2.0 * beta) / d.dx[ml];
      c[EC_BL] = bracket(d.dx[ml], h);
    } else {  // homogeneous Dirichlet face: u_hat = 0, full lift, mu_b
      c[EC_CL] = 2.0 / h;
      c[EC_CNL] = 0.0;
      c[EC_BL] = (1.0 + mu_star) * 2.0 / (h * r0);
    }
    if (hasr) {
      d.nbr[2 * m + 1] = mr;
      c[EC_CR] = (1.0 + 2.0 * beta) / h;
      c[EC_CNR] = (1.0 - 2.0 * beta) / d.dx[mr];
      c[EC_BR] = bracket(h, d.dx[mr]);
    } else {
      c[EC_CR] = 2.0 / h;
      c[EC_CNR] = 0.0;
      c[EC_BR] = (1.0 + mu_star) * 2.0 / (h * rP);
    }
  }
}

// Dense global 1D stiffness L_d (G x G, G = N * NP) from the element blocks.
void global_L(int P, const std::vector<double>& Ls, const std::vector<double>& D, const Dir1D& d,
              std::vector<double>& L) {
  const int NP = P + 1, N = d.N, G = N * NP;
  L.assign((size_t)G * G, 0.0);
  const double* D0 = &D[0];
  const double* DP = &D[P * NP];
  for (int m = 0; m < N; ++m) {
    const double* c = &d.ecoef[m * EC_COUNT];
    int r0 = m * NP;
    for (int i = 0; i < NP; ++i)
      for (int k = 0; k < NP; ++k) {
        double v = c[EC_TWO_DX] * Ls[i * NP + k];
        v += c[EC_CL] * (D0[i] * (k == 0) + (i == 0) * D0[k]) + c[EC_BL] * (i == 0) * (k == 0);
        v -= c[EC_CR] * (DP[i] * (k == P) + (i == P) * DP[k]);
        v += c[EC_BR] * (i == P) * (k == P);
        L[(size_t)(r0 + i) * G + r0 + k] += v;
      }
    int ml = d.nbr[2 * m], mr = d.nbr[2 * m + 1];
    if (ml >= 0)
      for (int i = 0; i < NP; ++i)
        for (int k = 0; k < NP; ++k) {
          double v = -c[EC_CL] * D0[i] * (k == P) + c[EC_CNL] * (i == 0) * DP[k] -
                     c[EC_BL] * (i == 0) * (k == P);
          L[(size_t)(r0 + i) * G + ml * NP + k] += v;
        }
    if (mr >= 0)
      for (int i = 0; i < NP; ++i)
        for (int k = 0; k < NP; ++k) {
          double v = c[EC_CR] * DP[i] * (k == 0) - c[EC_CNR] * (i == P) * D0[k] -
                     c[EC_BR] * (i == P) * (k == 0);
          L[(size_t)(r0 + i) * G + mr * NP + k] += v;
        }
  }
}

// Eigenpairs and weights of a 1D patch whose tile covers global indices
// start .. start + n - 1 (positions outside a Dirichlet domain are padding:
// identity eigenvector, eigenvalue 1, weight 0).
template <class WeightFn>
void patch_tables(int n, int start, int G, bool periodic, const std::vector<double>& L,
                  const std::vector<double>& mvec, WeightFn wfn, double* S, double* lam, double* w) {
  std::vector<int> pos, gidx;
  for (int t = 0; t < n; ++t) {
    int g = start + t;
    if (periodic) {
      pos.push_back(t);
      gidx.push_back(((g % G) + G) % G);
    } else if (g >= 0 && g < G) {
      pos.push_back(t);
      gidx.push_back(g);
    }
  }
  const int k = (int)pos.size();
  std::vector<double> Lk(k * k), mk(k), Sk, lk;
  for (int a = 0; a < k; ++a) {
    mk[a] = mvec[gidx[a]];
    for (int b = 0; b < k; ++b) Lk[a * k + b] = L[(size_t)gidx[a] * G + gidx[b]];
  }
  gen_eigen(k, Lk, mk, Sk, lk);
  for (int i = 0; i < n * n; ++i) S[i] = 0.0;
  for (int t = 0; t < n; ++t) {
    lam[t] = 1.0;
    w[t] = 0.0;
    S[t * n + t] = 1.0;
  }
  for (int a = 0; a < k; ++a) S[pos[a] * n + pos[a]] = 0.0;
  // eigenvector j of the valid block is stored in tile column pos[j]
  for (int a = 0; a < k; ++a)
    for (int j = 0; j < k; ++j) S[pos[a] * n + pos[j]] = Sk[a * k + j];
  for (int j = 0; j < k; ++j) lam[pos[j]] = lk[j];
  for (int a = 0; a < k; ++a) w[pos[a]] = wfn(start + pos[a]);
}

// Continuous spectral-element direction data (Sec. 4.3 counterpart): the
// assembled 1D stiffness L (dense nl x nl) and lumped mass of the stored
// lattice nodes (direct stiffness summation of (2/dx) L^s and (dx/2) rho).
void se_global_1d(int P, const std::vector<double>& Ls, const std::vector<double>& rho, const Dir1D& d,
                  std::vector<double>& L, std::vector<double>& mvec) {
  const int NP = P + 1, G = d.nl, NT = d.N * P;
  L.assign((size_t)G * G, 0.0);
  mvec.assign(G, 0.0);
  auto stored = [&](int g) {
    if (d.periodic) return ((g % NT) + NT) % NT;
    return (g >= 1 && g <= NT - 1) ? g - 1 : -1;
  };
  for (int m = 0; m < d.N; ++m) {
    const double h = d.dx[m];
    for (int i = 0; i < NP; ++i) {
      const int a = stored(m * P + i);
      if (a < 0) continue;
      mvec[a] += 0.5 * h * rho[i];
      for (int k = 0; k < NP; ++k) {
        const int b = stored(m * P + k);
        if (b >= 0) L[(size_t)a * G + b] += (2.0 / h) * Ls[i * NP + k];
      }
    }
  }
}

}  // namespace

std::string build_levels(const SetupParams& sp, std::vector<LevelHost>& levels) {
  std::vector<int> orders{sp.P};
  while (orders.back() > 1) orders.push_back(orders.back() / 2);
  std::reverse(orders.begin(), orders.end());
  levels.assign(orders.size(), LevelHost());
  for (size_t l = 0; l < orders.size(); ++l) {
    LevelHost& lv = levels[l];
    const int P = orders[l], NP = P + 1;
    lv.P = P;
    lv.NP = NP;
    lv.dim = sp.dim;
    const bool se = sp.disc == 1;
    lv.se = se;
    // continuous subdomains take N_O node layers of each neighbour beyond the
    // shared boundary node: the DG rule's value minus one (the DG subdomain
    // counts the coinciding neighbour node as a layer of its own)
    lv.NO = l == 0 ? 0 : overlap_rule(P, sp.overlap) - (se ? 1 : 0);
    if (lv.NO < 0 || lv.NO > P || (se && l > 0 && lv.NO + 1 > P)) {
      std::ostringstream os;
      if (se && lv.NO < 0) os << "continuous subdomains need the DG overlap N_O >= 1 on level P_l=" << P;
      else os << "overlap N_O=" << lv.NO << " outside [0, P_l=" << P << (se ? " - 1]" : "]");
      return os.str();
    }
    std::vector<double> eta;
    gll_points(P, eta, lv.rho);
    gll_diff(P, eta, lv.D);
    lv.Ls.assign(NP * NP, 0.0);
    for (int i = 0; i < NP; ++i)
      for (int k = 0; k < NP; ++k) {
        double s = 0.0;
        for (int j = 0; j < NP; ++j) s += lv.rho[j] * lv.D[j * NP + i] * lv.D[j * NP + k];
        lv.Ls[i * NP + k] = s;
      }
    lv.n_elem = 1;
    for (int d = 0; d < sp.dim; ++d) lv.n_elem *= sp.n[d];
    lv.n_dof = lv.n_elem;
    for (int d = 0; d < sp.dim; ++d) lv.n_dof *= NP;
    if (se) {
      lv.n_dof = 1;
      for (int d = 0; d < sp.dim; ++d) lv.n_dof *= sp.periodic[d] ? sp.n[d] * P : sp.n[d] * P - 1;
    }
    if (l > 0) {  // embedded interpolation from the coarser level (barycentric Lagrange)
      const int Pc = orders[l - 1], NPc = Pc + 1;
      std::vector<double> ec, rc;
      gll_points(Pc, ec, rc);
      std::vector<double> bw(NPc, 1.0);
      for (int k = 0; k < NPc; ++k)
        for (int j = 0; j < NPc; ++j)
          if (j != k) bw[k] /= (ec[k] - ec[j]);
      lv.NPc = NPc;
      lv.J.assign(NP * NPc, 0.0);
      for (int i = 0; i < NP; ++i) {
        int hit = -1;
        for (int k = 0; k < NPc; ++k)
          if (std::fabs(eta[i] - ec[k]) < 1e-15) hit = k;
        if (hit >= 0) {
          lv.J[i * NPc + hit] = 1.0;
          continue;
        }
        double den = 0.0;
        for (int k = 0; k < NPc; ++k) den += bw[k] / (eta[i] - ec[k]);
        for (int k = 0; k < NPc; ++k) lv.J[i * NPc + k] = bw[k] / (eta[i] - ec[k]) / den;
      }
    }
    for (int d = 0; d < sp.dim; ++d) {
      Dir1D& dd = lv.dir[d];
      dd.N = sp.n[d];
      dd.periodic = sp.periodic[d];
      dd.dx = sp.dx[d];
      const double beta = sp.flux == 1 ? sp.beta[d] : 0.0;
      element_coefficients(P, lv.rho, beta, sp.mu_star, dd);
      if (se) {
        dd.nl = dd.periodic ? dd.N * P : dd.N * P - 1;
        if (dd.nl < 1) return "a continuous Dirichlet direction needs at least one interior node";
        std::vector<double> L, mvec;
        se_global_1d(P, lv.Ls, lv.rho, dd, L, mvec);
        const int G = dd.nl;
        if (l == 0) {
          dd.G = G;
          gen_eigen(G, L, mvec, dd.S_glob, dd.lam_glob);
          dd.null_mode = -1;
          if (dd.periodic) {
            int imin = 0;
            for (int j = 0; j < G; ++j)
              if (std::fabs(dd.lam_glob[j]) < std::fabs(dd.lam_glob[imin])) imin = j;
            dd.null_mode = imin;
            dd.lam_glob[imin] = 0.0;
          }
          continue;
        }
        // element-centred subdomains: tile position t <-> lattice position m P - N_O + t
        const int NO = lv.NO;
        dd.n_ec = NP + 2 * NO;
        const int n = dd.n_ec;
        dd.S_ec.assign((size_t)dd.N * n * n, 0.0);
        dd.lam_ec.assign(dd.N * n, 0.0);
        dd.w_ec.assign(dd.N * n, 0.0);
        const double dxo = eta[NO + 1] + 1.0;  // distance to the nearest excluded node layer
        const int shift = dd.periodic ? 0 : 1;  // stored index = lattice position - shift
        for (int m = 0; m < dd.N; ++m) {
          const bool lb = !dd.periodic && m == 0, rb = !dd.periodic && m == dd.N - 1;
          auto wfn = [&](int gs) {
            const int g = gs + shift;
            int mm = (int)std::floor((double)g / P);
            int i = g - mm * P;
            double xh = eta[i] + 2.0 * (mm - m);
            double a = lb ? 1.0 : phi((1.0 + xh) / dxo, sp.weighting);
            double b = rb ? 1.0 : phi((1.0 - xh) / dxo, sp.weighting);
            return 0.5 * (a + b);
          };
          patch_tables(n, m * P - NO - shift, G, dd.periodic, L, mvec, wfn, &dd.S_ec[(size_t)m * n * n],
                       &dd.lam_ec[m * n], &dd.w_ec[m * n]);
        }
        continue;
      }
      std::vector<double> L, mvec(dd.N * NP);
      global_L(P, lv.Ls, lv.D, dd, L);
      for (int m = 0; m < dd.N; ++m)
        for (int i = 0; i < NP; ++i) mvec[m * NP + i] = 0.5 * dd.dx[m] * lv.rho[i];
      const int G = dd.N * NP;
      if (l == 0) {  // global eigenpairs for the exact coarse solve
        dd.G = G;
        gen_eigen(G, L, mvec, dd.S_glob, dd.lam_glob);
        dd.null_mode = -1;
        if (dd.periodic) {
          double lmax = 0;
          int imin = 0;
          for (int j = 0; j < G; ++j) {
            lmax = std::max(lmax, std::fabs(dd.lam_glob[j]));
            if (std::fabs(dd.lam_glob[j]) < std::fabs(dd.lam_glob[imin])) imin = j;
          }
          dd.null_mode = imin;
          dd.lam_glob[imin] = 0.0;
        }
        continue;
      }
      // element-centred patches
      const int NO = lv.NO;
      dd.n_ec = NP + 2 * NO;
      const int n = dd.n_ec;
      dd.S_ec.assign((size_t)dd.N * n * n, 0.0);
      dd.lam_ec.assign(dd.N * n, 0.0);
      dd.w_ec.assign(dd.N * n, 0.0);
      const double dxo = eta[NO] + 1.0;
      for (int m = 0; m < dd.N; ++m) {
        const bool lb = !dd.periodic && m == 0, rb = !dd.periodic && m == dd.N - 1;
        auto wfn = [&](int g) {
          if (NO == 0) return 1.0;
          int mm = (int)std::floor((double)g / NP);
          int i = g - mm * NP;
          double xh = eta[i] + 2.0 * (mm - m);
          double a = lb ? 1.0 : phi((1.0 + xh) / dxo, sp.weighting);
          double b = rb ? 1.0 : phi((1.0 - xh) / dxo, sp.weighting);
          return 0.5 * (a + b);
        };
        patch_tables(n, m * NP - NO, G, dd.periodic, L, mvec, wfn, &dd.S_ec[(size_t)m * n * n],
                     &dd.lam_ec[m * n], &dd.w_ec[m * n]);
      }
      // face-centred patches (normal direction)
      dd.nf = dd.periodic ? dd.N : dd.N + 1;
      dd.n_fc = 2 * P;
      const int a = dd.n_fc;
      dd.S_fc.assign((size_t)dd.nf * a * a, 0.0);
      dd.lam_fc.assign(dd.nf * a, 0.0);
      dd.w_fc.assign(dd.nf * a, 0.0);
      for (int f = 0; f < dd.nf; ++f) {
        auto wfn = [&](int g) {
          int mm = (int)std::floor((double)g / NP);
          int i = g - mm * NP;
          double xf = (mm == f - 1) ? eta[i] - 1.0 : eta[i] + 1.0;
          return 0.5 * (1.0 + phi(1.0 - std::fabs(xf), sp.weighting));
        };
        patch_tables(a, (f - 1) * NP + 1, G, dd.periodic, L, mvec, wfn, &dd.S_fc[(size_t)f * a * a],
                     &dd.lam_fc[f * a], &dd.w_fc[f * a]);
      }
    }
  }
  return std::string();
}

int face_count(const std::vector<LevelHost>& levels) {
  int c = 0;
  for (size_t l = 1; l < levels.size(); ++l)
    for (int d = 0; d < levels[l].dim; ++d) c += levels[l].dir[d].nf;
  return c;
}

void face_features(const std::vector<LevelHost>& levels, std::vector<double>& X) {
  X.clear();
  for (size_t l = 1; l < levels.size(); ++l) {
    const LevelHost& lv = levels[l];
    double mlog[3] = {0, 0, 0};
    for (int d = 0; d < lv.dim; ++d) {
      for (double h : lv.dir[d].dx) mlog[d] += std::log2(h);
      mlog[d] /= (double)lv.dir[d].dx.size();
    }
    for (int d = 0; d < lv.dim; ++d) {
      double lat = 0;
      for (int e = 0; e < lv.dim; ++e)
        if (e != d) lat += mlog[e];
      lat /= (double)(lv.dim - 1);
      const Dir1D& dd = lv.dir[d];
      for (int f = 0; f < dd.nf; ++f) {
        int left = f - 1, right = f;
        bool boundary = false;
        if (dd.periodic) {
          left = (left + dd.N) % dd.N;
          right = right % dd.N;
        } else {
          if (left < 0) left = 0, boundary = true;
          if (right >= dd.N) right = dd.N - 1, boundary = true;
        }
        X.push_back(lv.P / 32.0);
        X.push_back((std::log2(dd.dx[left]) - lat) / 5.0);
        X.push_back((std::log2(dd.dx[right]) - lat) / 5.0);
        X.push_back(boundary ? 1.0 : 0.0);
        X.push_back(lv.dim - 2.0);
        X.push_back(lv.NO / (double)lv.NP);
      }
    }
  }
}

void fc_weights_param(const LevelHost& lv, int d, int kind, const double* theta, const double* omega,
                      std::vector<double>& w) {
  const Dir1D& dd = lv.dir[d];
  const int NP = lv.NP, a = dd.n_fc, G = dd.N * NP;
  std::vector<double> eta, rho;
  gll_points(lv.P, eta, rho);
  w.assign((size_t)dd.nf * a, 0.0);
  std::vector<double> total(G, 0.0);
  std::vector<int> gi((size_t)dd.nf * a, -1);
  for (int f = 0; f < dd.nf; ++f)
    for (int t = 0; t < a; ++t) {
      const int g = (f - 1) * NP + 1 + t;
      int gw = g;
      if (dd.periodic) gw = ((g % G) + G) % G;
      else if (g < 0 || g >= G) continue;
      const int mm = (int)std::floor((double)g / NP), i = g - mm * NP;
      const double xf = (mm == f - 1) ? eta[i] - 1.0 : eta[i] + 1.0;
      const double wt = 0.5 * (1.0 + phi((1.0 - std::fabs(xf)) / theta[f], kind));
      w[(size_t)f * a + t] = wt;
      gi[(size_t)f * a + t] = gw;
      total[gw] += wt;
    }
  for (int f = 0; f < dd.nf; ++f)
    for (int t = 0; t < a; ++t) {
      const int gw = gi[(size_t)f * a + t];
      if (gw >= 0) w[(size_t)f * a + t] *= omega[f] / total[gw];
    }
}

}  // namespace dgmg

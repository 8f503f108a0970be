// Host FP64 trust-region step on the product manifold U(4)^P (or
// (U(2) x U(2))^P in parity mode), in an orthonormal tangent basis.
//
// Paper Sec. "Riemannian optimization": quadratic model
// m(X) = f + <grad f, X> + 1/2 <Hess f[X], X>, trust-region method with the
// truncated conjugate-gradient inner solver (Absil et al. Algorithms 10, 11;
// Steihaug), and the polar retraction R_V(xi) = q_polar(V + xi) per gate.
// The constants (theta = 1, kappa = 0.1, acceptance 0.1, radius factors 1/4
// and 2) are not given by the paper.
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "../../include/rq.h"

using cd = std::complex<double>;

namespace {

// Orthonormal basis A_mu of the anti-Hermitian 4x4 matrices:
// i E_aa (a = 0..3), (E_ab - E_ba)/sqrt2 and i (E_ab + E_ba)/sqrt2 for
// (a,b) in 01,02,03,12,13,23.  Parity mode: i E_00, i E_33,
// (E_03 - E_30)/sqrt2, i (E_03 + E_30)/sqrt2, i E_11, i E_22,
// (E_12 - E_21)/sqrt2, i (E_12 + E_21)/sqrt2.  Particle-number mode: the
// parity basis without the two (0,3) elements.
int basis(uint32_t flags, std::vector<cd> &B) {
  const bool parity = (flags & RQ_PARITY) != 0, number = (flags & RQ_NUMBER) != 0;
  const double r = std::sqrt(0.5);
  const cd I(0, 1);
  auto E = [](std::vector<cd> &M, int a, int b, cd v) { M[4 * a + b] += v; };
  B.clear();
  auto add = [&](std::vector<cd> M) { B.insert(B.end(), M.begin(), M.end()); };
  if (parity) {
    const int pr[2][2] = {{0, 3}, {1, 2}};
    for (int k = 0; k < 2; ++k) {
      const int a = pr[k][0], b = pr[k][1];
      std::vector<cd> M(16);
      E(M, a, a, I); add(M);
      M.assign(16, 0.0); E(M, b, b, I); add(M);
      if (number && k == 0) continue;
      M.assign(16, 0.0); E(M, a, b, r); E(M, b, a, -r); add(M);
      M.assign(16, 0.0); E(M, a, b, I * r); E(M, b, a, I * r); add(M);
    }
    return number ? 6 : 8;
  }
  for (int a = 0; a < 4; ++a) {
    std::vector<cd> M(16);
    E(M, a, a, I);
    add(M);
  }
  const int od[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  for (auto &p : od) {
    std::vector<cd> M(16);
    E(M, p[0], p[1], r);
    E(M, p[1], p[0], -r);
    add(M);
  }
  for (auto &p : od) {
    std::vector<cd> M(16);
    E(M, p[0], p[1], I * r);
    E(M, p[1], p[0], I * r);
    add(M);
  }
  return 16;
}

bool inv4(const cd *A, cd *Ai) {
  cd a[16], b[16];
  for (int i = 0; i < 16; ++i) {
    a[i] = A[i];
    b[i] = (i / 4 == i % 4) ? 1.0 : 0.0;
  }
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (std::abs(a[4 * r + c]) > std::abs(a[4 * piv + c])) piv = r;
    if (std::abs(a[4 * piv + c]) == 0.0) return false;
    for (int j = 0; j < 4; ++j) {
      std::swap(a[4 * piv + j], a[4 * c + j]);
      std::swap(b[4 * piv + j], b[4 * c + j]);
    }
    const cd d = 1.0 / a[4 * c + c];
    for (int j = 0; j < 4; ++j) {
      a[4 * c + j] *= d;
      b[4 * c + j] *= d;
    }
    for (int r = 0; r < 4; ++r) {
      if (r == c) continue;
      const cd f = a[4 * r + c];
      for (int j = 0; j < 4; ++j) {
        a[4 * r + j] -= f * a[4 * c + j];
        b[4 * r + j] -= f * b[4 * c + j];
      }
    }
  }
  for (int i = 0; i < 16; ++i) Ai[i] = b[i];
  return true;
}

// Unitary polar factor by the Newton iteration X <- (X + X^{-dagger}) / 2,
// which converges quadratically to Q for nonsingular A = Q P (Higham).
bool polar4(const cd *A, cd *Q) {
  cd X[16], Xi[16];
  for (int i = 0; i < 16; ++i) X[i] = A[i];
  for (int it = 0; it < 100; ++it) {
    if (!inv4(X, Xi)) return false;
    double diff = 0.0;
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        const cd nx = 0.5 * (X[4 * i + j] + std::conj(Xi[4 * j + i]));
        diff += std::norm(nx - X[4 * i + j]);
        Q[4 * i + j] = nx;
      }
    for (int i = 0; i < 16; ++i) X[i] = Q[i];
    if (diff < 1e-30) break;
  }
  return true;
}

}  // namespace

extern "C" {

int rq_tangent_basis(uint32_t flags, double *out) {
  std::vector<cd> B;
  const int d = basis(flags, B);
  if (out)
    for (int i = 0; i < d * 16; ++i) {
      out[2 * i] = B[i].real();
      out[2 * i + 1] = B[i].imag();
    }
  return d;
}

int rq_tr_step(int32_t n_params, uint32_t flags, const double *gates, const double *g,
               const double *H, double delta, double *eta, double *cand,
               double *model_decrease, int32_t *stop) {
  if (n_params < 1 || !gates || !g || !H || !eta || !cand || !(delta > 0)) return RQ_EINVAL;
  std::vector<cd> B;
  const int d = basis(flags, B);
  const int n = n_params * d;
  auto dot = [n](const double *a, const double *b) {
    double s = 0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
  };
  auto matvec = [&](const double *x, double *y) {
    for (int i = 0; i < n; ++i) {
      double s = 0;
      const double *row = H + size_t(i) * n;
      for (int j = 0; j < n; ++j) s += row[j] * x[j];
      y[i] = s;
    }
  };
  // truncated CG (Steihaug-Toint), theta = 1, kappa = 0.1
  std::vector<double> r(g, g + n), dl(n), Hd(n), e(n, 0.0), en(n);
  for (int i = 0; i < n; ++i) dl[i] = -r[i];
  const double r0 = std::sqrt(dot(r.data(), r.data()));
  int why = 3;
  auto to_boundary = [&](const std::vector<double> &x, const std::vector<double> &dd) {
    const double a = dot(dd.data(), dd.data()), b = 2 * dot(x.data(), dd.data()),
                 c = dot(x.data(), x.data()) - delta * delta;
    const double tau = (-b + std::sqrt(b * b - 4 * a * c)) / (2 * a);
    for (int i = 0; i < n; ++i) e[i] = x[i] + tau * dd[i];
  };
  if (r0 == 0.0) {
    why = 4;
  } else {
    double rr = dot(r.data(), r.data());
    for (int it = 0; it < n; ++it) {
      matvec(dl.data(), Hd.data());
      const double dHd = dot(dl.data(), Hd.data());
      if (dHd <= 0) {
        to_boundary(std::vector<double>(e), dl);
        why = 2;
        break;
      }
      const double alpha = rr / dHd;
      for (int i = 0; i < n; ++i) en[i] = e[i] + alpha * dl[i];
      if (std::sqrt(dot(en.data(), en.data())) >= delta) {
        to_boundary(std::vector<double>(e), dl);
        why = 1;
        break;
      }
      e = en;
      for (int i = 0; i < n; ++i) r[i] += alpha * Hd[i];
      const double rrn = dot(r.data(), r.data());
      if (std::sqrt(rrn) <= r0 * std::min(r0, 0.1)) {
        why = 0;
        break;
      }
      for (int i = 0; i < n; ++i) dl[i] = -r[i] + (rrn / rr) * dl[i];
      rr = rrn;
    }
  }
  for (int i = 0; i < n; ++i) eta[i] = e[i];
  std::vector<double> He(n);
  matvec(e.data(), He.data());
  if (model_decrease) *model_decrease = -(dot(g, e.data()) + 0.5 * dot(e.data(), He.data()));
  if (stop) *stop = why;
  // retraction per gate: polar(G_p + G_p sum_mu eta A_mu)
  for (int p = 0; p < n_params; ++p) {
    cd G[16], A[16], X[16], Q[16];
    for (int i = 0; i < 16; ++i) {
      G[i] = cd(gates[(size_t(p) * 16 + i) * 2], gates[(size_t(p) * 16 + i) * 2 + 1]);
      A[i] = 0.0;
    }
    for (int m = 0; m < d; ++m)
      for (int i = 0; i < 16; ++i) A[i] += e[size_t(p) * d + m] * B[size_t(m) * 16 + i];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        cd s = 0;
        for (int k = 0; k < 4; ++k) s += G[4 * i + k] * A[4 * k + j];
        X[4 * i + j] = G[4 * i + j] + s;
      }
    if (!polar4(X, Q)) return RQ_ESINGULAR;
    for (int i = 0; i < 16; ++i) {
      cand[(size_t(p) * 16 + i) * 2] = Q[i].real();
      cand[(size_t(p) * 16 + i) * 2 + 1] = Q[i].imag();
    }
  }
  return RQ_OK;
}

int rq_tangent_coords(int32_t n_params, uint32_t flags, const double *gates, const double *Y,
                      double *out) {
  if (n_params < 1 || !gates || !Y || !out) return RQ_EINVAL;
  std::vector<cd> B;
  const int d = basis(flags, B);
  for (int p = 0; p < n_params; ++p) {
    cd G[16], Yp[16];
    for (int i = 0; i < 16; ++i) {
      G[i] = cd(gates[(size_t(p) * 16 + i) * 2], gates[(size_t(p) * 16 + i) * 2 + 1]);
      Yp[i] = cd(Y[(size_t(p) * 16 + i) * 2], Y[(size_t(p) * 16 + i) * 2 + 1]);
    }
    for (int m = 0; m < d; ++m) {
      // <G A_m, Y> = Re sum_ab conj((G A_m)_ab) Y_ab
      double s = 0.0;
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          cd x = 0.0;
          for (int c = 0; c < 4; ++c) x += G[4 * a + c] * B[size_t(m) * 16 + 4 * c + b];
          s += (std::conj(x) * Yp[4 * a + b]).real();
        }
      out[size_t(p) * d + m] = s;
    }
  }
  return RQ_OK;
}

int rq_tr_accept(double f0, double f1, double model_decrease, double delta, double delta_bar,
                 double eta_norm, double *new_delta, int32_t *accepted, double *rho) {
  if (!new_delta || !accepted) return RQ_EINVAL;
  const double r = model_decrease > 0 ? (f0 - f1) / model_decrease : -INFINITY;
  const bool on_boundary = std::fabs(eta_norm - delta) <= 1e-12 * std::max(1.0, delta);
  double nd = delta;
  if (r < 0.25)
    nd = 0.25 * delta;
  else if (r > 0.75 && on_boundary)
    nd = std::min(2 * delta, delta_bar);
  *new_delta = nd;
  *accepted = r > 0.1;
  if (rho) *rho = r;
  return RQ_OK;
}

}  // extern "C"

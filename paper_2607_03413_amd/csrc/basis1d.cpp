// 1D reference data on [0, 1]: Gauss-Lobatto nodes, Lagrange basis, mass and
// stiffness matrices, the two child prolongation matrices, and a small dense
// symmetric generalized eigensolver.  Host code, FP64.
//
// Paper: continuous Q_p with a Gauss-Lobatto nodal basis (Sec. 2); transfers
// by the 1D matrices P_0, P_1 of the two children (Sec. 3.1).
#include <algorithm>
#include <cmath>

#include "fe_internal.h"

namespace fe {

namespace {
// Legendre P_n and P_n' at x in [-1, 1].
void legendre(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) { p = 1.0; dp = 0.0; return; }
  for (int m = 1; m < n; ++m) {
    double p2 = ((2.0 * m + 1.0) * x * p1 - m * p0) / (m + 1.0);
    double d2 = d0 + (2.0 * m + 1.0) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  p = p1; dp = d1;
}
}  // namespace

std::vector<double> gll_nodes(int k) {
  // Interior nodes: roots of P_k'.  Newton on q = (1-x^2) P_k' with q' = -k(k+1) P_k.
  std::vector<double> t(k + 1);
  for (int j = 0; j <= k; ++j) t[j] = -std::cos(M_PI * j / k);
  for (int j = 1; j < k; ++j) {
    double x = t[j];
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(k, x, p, dp);
      double step = (1.0 - x * x) * dp / (-k * (k + 1.0) * p);
      x -= step;
      if (std::fabs(step) < 1e-17) break;
    }
    t[j] = x;
  }
  t[0] = -1.0; t[k] = 1.0;
  std::vector<double> out(k + 1);
  for (int j = 0; j <= k; ++j) out[j] = 0.5 * (t[j] + 1.0);
  return out;
}

void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0); w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double p = 0.0, dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      legendre(n, t, p, dp);
      double step = p / dp;
      t -= step;
      if (std::fabs(step) < 1e-17) break;
    }
    legendre(n, t, p, dp);
    x[n - 1 - i] = 0.5 * (t + 1.0);
    w[n - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp);   // 2/((1-t^2)P'^2) on [-1,1], halved
  }
}

double lagrange_value(const std::vector<double>& nodes, int j, double x) {
  double v = 1.0;
  for (size_t m = 0; m < nodes.size(); ++m)
    if ((int)m != j) v *= (x - nodes[m]) / (nodes[j] - nodes[m]);
  return v;
}

double lagrange_deriv(const std::vector<double>& nodes, int j, double x) {
  double s = 0.0;
  const int n = (int)nodes.size();
  for (int l = 0; l < n; ++l) {
    if (l == j) continue;
    double t = 1.0 / (nodes[j] - nodes[l]);
    for (int m = 0; m < n; ++m)
      if (m != j && m != l) t *= (x - nodes[m]) / (nodes[j] - nodes[m]);
    s += t;
  }
  return s;
}

static std::vector<double> integrate_pairs(int k, bool deriv) {
  const int K = k + 1;
  std::vector<double> nodes = gll_nodes(k), xq, wq;
  gauss_rule(K, xq, wq);
  std::vector<double> out(K * K, 0.0);
  for (int q = 0; q < K; ++q) {
    double v[kMaxK];
    for (int j = 0; j < K; ++j)
      v[j] = deriv ? lagrange_deriv(nodes, j, xq[q]) : lagrange_value(nodes, j, xq[q]);
    for (int i = 0; i < K; ++i)
      for (int j = 0; j < K; ++j) out[i * K + j] += wq[q] * v[i] * v[j];
  }
  return out;
}

std::vector<double> mass_1d(int k) { return integrate_pairs(k, false); }
std::vector<double> stiffness_1d(int k) { return integrate_pairs(k, true); }

std::vector<double> prolongation_1d(int k, int c) {
  const int K = k + 1;
  std::vector<double> nodes = gll_nodes(k), out(K * K);
  for (int i = 0; i < K; ++i)
    for (int j = 0; j < K; ++j) out[i * K + j] = lagrange_value(nodes, j, 0.5 * (nodes[i] + c));
  return out;
}

bool sym_generalized_eig(int n, const std::vector<double>& A, const std::vector<double>& M,
                         std::vector<double>& S, std::vector<double>& lam) {
  // Cholesky M = L L^T
  std::vector<double> L(n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = M[j * n + j];
    for (int p = 0; p < j; ++p) d -= L[j * n + p] * L[j * n + p];
    if (!(d > 0.0)) return false;
    L[j * n + j] = std::sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double s = M[i * n + j];
      for (int p = 0; p < j; ++p) s -= L[i * n + p] * L[j * n + p];
      L[i * n + j] = s / L[j * n + j];
    }
  }
  // Linv by forward substitution
  std::vector<double> Li(n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int p = 0; p < i; ++p) s -= L[i * n + p] * Li[p * n + c];
      Li[i * n + c] = s / L[i * n + i];
    }
  }
  // C = Linv A Linv^T
  std::vector<double> T(n * n, 0.0), C(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int p = 0; p < n; ++p) s += Li[i * n + p] * A[p * n + j];
      T[i * n + j] = s;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int p = 0; p < n; ++p) s += T[i * n + p] * Li[j * n + p];
      C[i * n + j] = s;
    }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) C[i * n + j] = C[j * n + i] = 0.5 * (C[i * n + j] + C[j * n + i]);
  // cyclic Jacobi: C = Q diag Q^T
  std::vector<double> Q(n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += C[i * n + j] * C[i * n + j];
        if (i != j) off += C[i * n + j] * C[i * n + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = C[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double theta = (C[q * n + q] - C[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < n; ++r) {  // columns p, q
          double crp = C[r * n + p], crq = C[r * n + q];
          C[r * n + p] = c * crp - s * crq;
          C[r * n + q] = s * crp + c * crq;
        }
        for (int r = 0; r < n; ++r) {  // rows p, q
          double cpr = C[p * n + r], cqr = C[q * n + r];
          C[p * n + r] = c * cpr - s * cqr;
          C[q * n + r] = s * cpr + c * cqr;
        }
        for (int r = 0; r < n; ++r) {
          double qrp = Q[r * n + p], qrq = Q[r * n + q];
          Q[r * n + p] = c * qrp - s * qrq;
          Q[r * n + q] = s * qrp + c * qrq;
        }
      }
  }
  // sort ascending, S = Linv^T Q
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return C[a * n + a] < C[b * n + b]; });
  lam.assign(n, 0.0);
  S.assign(n * n, 0.0);
  for (int jj = 0; jj < n; ++jj) {
    int j = ord[jj];
    lam[jj] = C[j * n + j];
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int p = 0; p < n; ++p) s += Li[p * n + i] * Q[p * n + j];
      S[i * n + jj] = s;
    }
  }
  return true;
}

}  // namespace fe

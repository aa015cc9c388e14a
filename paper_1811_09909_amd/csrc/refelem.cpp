// Reference element of the HDG discretization (host side, built once per
// problem): GLL-nodal Q^k bases on a cell of size h, Gauss rules with k+2
// points per direction, and the element integrals that enter the local
// problems of eqs. HDG and HDG_flux and of the hybridized IPDG family
// (eq. IPG_H).
#include <cmath>
#include <stdexcept>

#include "hdg_internal.hpp"

namespace hdg {

namespace {

// Legendre P_n(x) and P_n'(x) by the three-term recurrence (long double).
void legendre(int n, long double x, long double& p, long double& dp) {
  long double p0 = 1.0L, p1 = x;
  if (n == 0) {
    p = 1.0L;
    dp = 0.0L;
    return;
  }
  for (int m = 2; m <= n; ++m) {
    long double p2 = ((2 * m - 1) * x * p1 - (m - 1) * p0) / m;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  // n P_{n-1} = n x P_n + (1 - x^2) P_n'  ->  P_n' = n (P_{n-1} - x P_n) / (1 - x^2)
  dp = n * (p0 - x * p1) / (1.0L - x * x);
}

long double lagrange_value(const std::vector<double>& xi, int i, long double t) {
  long double v = 1.0L;
  for (size_t j = 0; j < xi.size(); ++j)
    if ((int)j != i) v *= (t - xi[j]) / ((long double)xi[i] - xi[j]);
  return v;
}

long double lagrange_deriv(const std::vector<double>& xi, int i, long double t) {
  long double s = 0.0L;
  for (size_t m = 0; m < xi.size(); ++m) {
    if ((int)m == i) continue;
    long double term = 1.0L / ((long double)xi[i] - xi[m]);
    for (size_t j = 0; j < xi.size(); ++j)
      if ((int)j != i && j != m) term *= (t - xi[j]) / ((long double)xi[i] - xi[j]);
    s += term;
  }
  return s;
}

}  // namespace

void gll_points(int k, std::vector<double>& out) {
  // end points plus the k-1 roots of P_k' on [-1,1], found by Newton's method
  // on P_k' with P_k'' from the Legendre equation; mapped to [0,1].
  std::vector<long double> x(k + 1);
  x[0] = -1.0L;
  x[k] = 1.0L;
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int j = 1; j < k; ++j) {
    long double t = -std::cos(pi * j / k);
    for (int it = 0; it < 100; ++it) {
      long double p, dp;
      legendre(k, t, p, dp);
      long double d2p = (2.0L * t * dp - k * (k + 1.0L) * p) / (1.0L - t * t);
      long double dt = dp / d2p;
      t -= dt;
      if (std::fabs(dt) < 1e-19L) break;
    }
    x[j] = t;
  }
  out.resize(k + 1);
  for (int j = 0; j <= k; ++j) out[j] = (double)(0.5L * (x[j] + 1.0L));
  out[0] = 0.0;
  out[k] = 1.0;
}

void gauss_points(int n, std::vector<double>& xo, std::vector<double>& wo) {
  const long double pi = 3.141592653589793238462643383279502884L;
  xo.resize(n);
  wo.resize(n);
  for (int i = 0; i < n; ++i) {
    long double t = -std::cos(pi * (i + 0.75L) / (n + 0.5L));
    long double p, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(n, t, p, dp);
      long double dt = p / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-19L) break;
    }
    legendre(n, t, p, dp);
    long double w = 2.0L / ((1.0L - t * t) * dp * dp);
    xo[i] = (double)(0.5L * (t + 1.0L));
    wo[i] = (double)(0.5L * w);
  }
}

void RefElement::build(int d_, int k_, double h_) {
  d = d_;
  k = k_;
  h = h_;
  const int p1 = k + 1, q1 = k + 2;
  nv = 1;
  ne = 1;
  nq = 1;
  for (int i = 0; i < d; ++i) {
    nv *= p1;
    nq *= q1;
  }
  for (int i = 0; i < d - 1; ++i) ne *= p1;
  nc = 1 << (d - 1);
  nf = 2 * d;
  nl = nf * ne;
  gll_points(k, gll);
  gauss_points(q1, gauss, gw);

  // 1D tables: l[i][q] = l_i(g_q), dl[i][q] = l_i'(g_q), end[i][side] = l_i(side)
  std::vector<double> l(p1 * q1), dl(p1 * q1), end(p1 * 2);
  for (int i = 0; i < p1; ++i) {
    for (int q = 0; q < q1; ++q) {
      l[i * q1 + q] = (double)lagrange_value(gll, i, gauss[q]);
      dl[i * q1 + q] = (double)(lagrange_deriv(gll, i, gauss[q]) / h);
    }
    end[i * 2 + 0] = (i == 0) ? 1.0 : 0.0;
    end[i * 2 + 1] = (i == k) ? 1.0 : 0.0;
  }
  auto digit = [](int idx, int base, int pos) {
    for (int t = 0; t < pos; ++t) idx /= base;
    return idx % base;
  };

  // volume quadrature
  Phi.assign((size_t)nq * nv, 1.0);
  Wq.assign(nq, 1.0);
  std::vector<double> dPhi((size_t)d * nq * nv, 1.0);
  double hd = std::pow(h, d);
  for (int Q = 0; Q < nq; ++Q) {
    double w = hd;
    for (int a = 0; a < d; ++a) w *= gw[digit(Q, q1, a)];
    Wq[Q] = w;
    for (int I = 0; I < nv; ++I) {
      double v = 1.0;
      for (int a = 0; a < d; ++a) v *= l[digit(I, p1, a) * q1 + digit(Q, q1, a)];
      Phi[(size_t)Q * nv + I] = v;
      for (int c = 0; c < d; ++c) {
        double g = 1.0;
        for (int a = 0; a < d; ++a) {
          int i = digit(I, p1, a), q = digit(Q, q1, a);
          g *= (a == c) ? dl[i * q1 + q] : l[i * q1 + q];
        }
        dPhi[((size_t)c * nq + Q) * nv + I] = g;
      }
    }
  }
  M.assign((size_t)nv * nv, 0.0);
  B.assign((size_t)d * nv * nv, 0.0);
  for (int i = 0; i < nv; ++i)
    for (int j = 0; j < nv; ++j) {
      double s = 0.0;
      for (int Q = 0; Q < nq; ++Q) s += Wq[Q] * Phi[(size_t)Q * nv + i] * Phi[(size_t)Q * nv + j];
      M[(size_t)i * nv + j] = s;
      for (int c = 0; c < d; ++c) {
        double b = 0.0;
        for (int Q = 0; Q < nq; ++Q)
          b += Wq[Q] * dPhi[((size_t)c * nq + Q) * nv + j] * Phi[(size_t)Q * nv + i];
        B[((size_t)c * nv + i) * nv + j] = b;
      }
    }

  // stiffness K[i][j] = (grad phi_j, grad phi_i) of the primal IPDG forms
  Kst.assign((size_t)nv * nv, 0.0);
  for (int i = 0; i < nv; ++i)
    for (int j = 0; j < nv; ++j) {
      double s = 0.0;
      for (int c = 0; c < d; ++c)
        for (int Q = 0; Q < nq; ++Q)
          s += Wq[Q] * dPhi[((size_t)c * nq + Q) * nv + i] * dPhi[((size_t)c * nq + Q) * nv + j];
      Kst[(size_t)i * nv + j] = s;
    }
  // derivatives of the basis at its own nodes: Dnode[c][a][j] = d_c phi_j(x_a)
  Dnode.assign((size_t)d * nv * nv, 0.0);
  for (int c = 0; c < d; ++c)
    for (int a = 0; a < nv; ++a)
      for (int j = 0; j < nv; ++j) {
        double v = 1.0;
        for (int b = 0; b < d; ++b) {
          const int ja = digit(j, p1, b), aa = digit(a, p1, b);
          v *= (b == c) ? (double)(lagrange_deriv(gll, ja, gll[aa]) / h) : (ja == aa ? 1.0 : 0.0);
        }
        Dnode[((size_t)c * nv + a) * nv + j] = v;
      }

  // face quadrature: tangential Gauss points of each face slot
  int nfq = 1;
  for (int i = 0; i < d - 1; ++i) nfq *= q1;
  double hf = std::pow(h, d - 1);
  F.assign((size_t)d * nv * nl, 0.0);
  G.assign((size_t)nv * nl, 0.0);
  E.assign((size_t)nv * nv, 0.0);
  H.assign((size_t)nl * nl, 0.0);
  Nn.assign((size_t)nv * nv, 0.0);
  Dn.assign((size_t)nv * nl, 0.0);
  std::vector<double> pf((size_t)nfq * nv), mu((size_t)nfq * ne), wf(nfq), dpf((size_t)nfq * nv);
  for (int s = 0; s < nf; ++s) {
    int c = s / 2, side = s % 2;
    double nrm = side ? 1.0 : -1.0;
    int tang[2] = {0, 0}, nt = 0;
    for (int a = 0; a < d; ++a)
      if (a != c) tang[nt++] = a;
    for (int P = 0; P < nfq; ++P) {
      double w = hf;
      for (int j = 0; j < d - 1; ++j) w *= gw[digit(P, q1, j)];
      wf[P] = w;
      for (int m = 0; m < ne; ++m) {
        double v = 1.0;
        for (int j = 0; j < d - 1; ++j) v *= l[digit(m, p1, j) * q1 + digit(P, q1, j)];
        mu[(size_t)P * ne + m] = v;
      }
      for (int I = 0; I < nv; ++I) {
        double v = end[digit(I, p1, c) * 2 + side];
        for (int j = 0; j < d - 1; ++j) v *= l[digit(I, p1, tang[j]) * q1 + digit(P, q1, j)];
        pf[(size_t)P * nv + I] = v;
        // outward normal derivative n_c d_c phi_I at the face point
        double g = nrm * (double)(lagrange_deriv(gll, digit(I, p1, c), (long double)side) / h);
        for (int j = 0; j < d - 1; ++j) g *= l[digit(I, p1, tang[j]) * q1 + digit(P, q1, j)];
        dpf[(size_t)P * nv + I] = g;
      }
    }
    for (int i = 0; i < nv; ++i) {
      for (int m = 0; m < ne; ++m) {
        double g = 0.0;
        for (int P = 0; P < nfq; ++P) g += wf[P] * mu[(size_t)P * ne + m] * pf[(size_t)P * nv + i];
        G[(size_t)i * nl + s * ne + m] = g;
        F[((size_t)c * nv + i) * nl + s * ne + m] = nrm * g;
      }
      for (int j = 0; j < nv; ++j) {
        double e = 0.0, nn = 0.0;
        for (int P = 0; P < nfq; ++P) {
          e += wf[P] * pf[(size_t)P * nv + i] * pf[(size_t)P * nv + j];
          nn += wf[P] * dpf[(size_t)P * nv + i] * pf[(size_t)P * nv + j];
        }
        E[(size_t)i * nv + j] += e;
        Nn[(size_t)i * nv + j] += nn;
      }
      for (int m = 0; m < ne; ++m) {
        double v = 0.0;
        for (int P = 0; P < nfq; ++P) v += wf[P] * dpf[(size_t)P * nv + i] * mu[(size_t)P * ne + m];
        Dn[(size_t)i * nl + s * ne + m] = v;
      }
    }
    for (int m = 0; m < ne; ++m)
      for (int mm = 0; mm < ne; ++mm) {
        double v = 0.0;
        for (int P = 0; P < nfq; ++P) v += wf[P] * mu[(size_t)P * ne + m] * mu[(size_t)P * ne + mm];
        H[(size_t)(s * ne + m) * nl + s * ne + mm] = v;
      }
  }

  // P1 (Q1) vertex basis of a face evaluated at its GLL nodes
  Jp.assign((size_t)ne * nc, 1.0);
  for (int a = 0; a < ne; ++a)
    for (int v = 0; v < nc; ++v) {
      double w = 1.0;
      for (int j = 0; j < d - 1; ++j) {
        double t = gll[digit(a, p1, j)];
        w *= ((v >> j) & 1) ? t : 1.0 - t;
      }
      Jp[(size_t)a * nc + v] = w;
    }
}

// Raviart-Thomas data of the hybridized mixed method (eqs. mixed_local1/2)
// on squares (d = 2): RT_k = Q_{k+1,k} x Q_{k,k+1}, each component nodal at
// tensor GLL points of degree k+1 along its own direction and k across it
// (x fastest), velocity coefficients ordered [x component, y component].
void RefElement::build_rt() {
  if (d != 2) throw std::invalid_argument("RT-H is two-dimensional");
  const int p1 = k + 1, q1 = k + 2;
  std::vector<double> ghi;
  gll_points(k + 1, ghi);
  nqc = (k + 2) * (k + 1);
  nqv = 2 * nqc;
  // 1D tables: degree k+1 basis (k+2 functions) and degree k basis (k+1)
  std::vector<double> lhi((size_t)(k + 2) * q1), dlhi((size_t)(k + 2) * q1), llo((size_t)p1 * q1);
  std::vector<double> hiend((size_t)(k + 2) * 2), hinode((size_t)(k + 2) * p1);
  for (int i = 0; i < k + 2; ++i) {
    for (int q = 0; q < q1; ++q) {
      lhi[i * q1 + q] = (double)lagrange_value(ghi, i, gauss[q]);
      dlhi[i * q1 + q] = (double)(lagrange_deriv(ghi, i, gauss[q]) / h);
    }
    hiend[i * 2 + 0] = i == 0 ? 1.0 : 0.0;
    hiend[i * 2 + 1] = i == k + 1 ? 1.0 : 0.0;
    for (int a = 0; a < p1; ++a) hinode[i * p1 + a] = (double)lagrange_value(ghi, i, gll[a]);
  }
  for (int i = 0; i < p1; ++i)
    for (int q = 0; q < q1; ++q) llo[i * q1 + q] = (double)lagrange_value(gll, i, gauss[q]);
  // basis index I of component c -> (a_0, a_1), degree k+1 along c
  auto split = [&](int c, int I, int* a) {
    const int n0 = c == 0 ? k + 2 : p1;
    a[0] = I % n0;
    a[1] = I / n0;
  };
  Vq.assign((size_t)2 * nq * nqc, 0.0);
  std::vector<double> Dq((size_t)2 * nq * nqc, 0.0);
  for (int c = 0; c < 2; ++c)
    for (int Q = 0; Q < nq; ++Q) {
      const int qd[2] = {Q % q1, Q / q1};
      for (int I = 0; I < nqc; ++I) {
        int a[2];
        split(c, I, a);
        double v = 1.0, g = 1.0;
        for (int t = 0; t < 2; ++t) {
          v *= t == c ? lhi[a[t] * q1 + qd[t]] : llo[a[t] * q1 + qd[t]];
          g *= t == c ? dlhi[a[t] * q1 + qd[t]] : llo[a[t] * q1 + qd[t]];
        }
        Vq[((size_t)c * nq + Q) * nqc + I] = v;
        Dq[((size_t)c * nq + Q) * nqc + I] = g;
      }
    }
  // Bd[c*nqc + I][j] = (phi_j, div v_I)
  Bd.assign((size_t)nqv * nv, 0.0);
  for (int c = 0; c < 2; ++c)
    for (int I = 0; I < nqc; ++I)
      for (int j = 0; j < nv; ++j) {
        double sum = 0.0;
        for (int Q = 0; Q < nq; ++Q) sum += Wq[Q] * Dq[((size_t)c * nq + Q) * nqc + I] * Phi[(size_t)Q * nv + j];
        Bd[((size_t)c * nqc + I) * nv + j] = sum;
      }
  // Fr[c*nqc + I][s*ne + m] = <mu_m, v_I . n> on face slot s = 2 cc + side
  Fr.assign((size_t)nqv * nl, 0.0);
  for (int s = 0; s < nf; ++s) {
    const int cc = s / 2, side = s % 2, tg = 1 - cc;
    const double nrm = side ? 1.0 : -1.0;
    for (int I = 0; I < nqc; ++I) {
      int a[2];
      split(cc, I, a);
      for (int m = 0; m < ne; ++m) {
        double sum = 0.0;
        for (int P = 0; P < q1; ++P) {
          const double v = hiend[a[cc] * 2 + side] * llo[a[tg] * q1 + P];
          const double mu = (double)lagrange_value(gll, m, gauss[P]);
          sum += h * gw[P] * v * mu;
        }
        Fr[((size_t)cc * nqc + I) * nl + s * ne + m] = nrm * sum;
      }
    }
  }
  // Vnode[c][a][I] = v_{c,I} at the scalar's node a
  Vnode.assign((size_t)2 * nv * nqc, 0.0);
  for (int c = 0; c < 2; ++c)
    for (int A = 0; A < nv; ++A) {
      const int na[2] = {A % p1, A / p1};
      for (int I = 0; I < nqc; ++I) {
        int a[2];
        split(c, I, a);
        double v = 1.0;
        for (int t = 0; t < 2; ++t) v *= t == c ? hinode[a[t] * p1 + na[t]] : (a[t] == na[t] ? 1.0 : 0.0);
        Vnode[((size_t)c * nv + A) * nqc + I] = v;
      }
    }
}

}  // namespace hdg

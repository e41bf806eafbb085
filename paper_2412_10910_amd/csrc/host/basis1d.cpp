// 1D tables of the Q_k element: Gauss-Legendre quadrature (k+1 points, paper §4)
// and Lagrange polynomials on the Gauss-Lobatto support points (paper §3.2).
#include <cmath>

#include "../internal.hpp"

namespace nnmg {
namespace {

using real = long double;
const real kPi = 3.141592653589793238462643383279502884L;

// Legendre P_m and its derivative at x by the three-term recurrence
void legendre(int m, real x, real& p, real& dp) {
    real p0 = 1, p1 = x;
    if (m == 0) {
        p = 1;
        dp = 0;
        return;
    }
    for (int j = 2; j <= m; ++j) {
        real p2 = ((2 * j - 1) * x * p1 - (j - 1) * p0) / j;
        p0 = p1;
        p1 = p2;
    }
    p = p1;
    dp = m * (x * p1 - p0) / (x * x - 1);
}

real lagrange(const real* x, int n, int a, real t) {
    real v = 1;
    for (int m = 0; m < n; ++m)
        if (m != a) v *= (t - x[m]) / (x[a] - x[m]);
    return v;
}

real lagrange_deriv(const real* x, int n, int a, real t) {
    real s = 0;
    for (int l = 0; l < n; ++l) {
        if (l == a) continue;
        real term = 1 / (x[a] - x[l]);
        for (int m = 0; m < n; ++m)
            if (m != a && m != l) term *= (t - x[m]) / (x[a] - x[m]);
        s += term;
    }
    return s;
}

}  // namespace

Basis1D make_basis(int degree) {
    Basis1D b;
    const int n = degree + 1;
    b.n = n;
    real g[kMaxN], w[kMaxN], xn[kMaxN];
    // Gauss-Legendre: Newton on P_n from the classical initial guesses
    for (int i = 0; i < n; ++i) {
        real x = -std::cos(kPi * (i + 0.75L) / (n + 0.5L));
        for (int it = 0; it < 100; ++it) {
            real p, dp;
            legendre(n, x, p, dp);
            real dx = p / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-30L) break;
        }
        real p, dp;
        legendre(n, x, p, dp);
        g[i] = (x + 1) / 2;
        w[i] = 1 / ((1 - x * x) * dp * dp);  // 2/((1-x^2)P'^2) scaled by 1/2 for [0,1]
    }
    // Gauss-Lobatto: end points and the roots of P_k'
    xn[0] = 0;
    xn[degree] = 1;
    for (int j = 1; j < degree; ++j) {
        real x = -std::cos(kPi * j / degree);
        for (int it = 0; it < 100; ++it) {
            real p, dp;
            legendre(degree, x, p, dp);
            // P'' from the Legendre equation (1-x^2) P'' - 2x P' + k(k+1) P = 0
            real d2p = (2 * x * dp - degree * (degree + 1) * p) / (1 - x * x);
            real dx = dp / d2p;
            x -= dx;
            if (std::fabs(dx) < 1e-30L) break;
        }
        xn[j] = (x + 1) / 2;
    }
    for (int i = 0; i < n; ++i) {
        b.gauss[i] = (double)g[i];
        b.weight[i] = (double)w[i];
        b.node[i] = (double)xn[i];
        real pr = 1;
        for (int m = 0; m < n; ++m)
            if (m != i) pr *= xn[i] - xn[m];
        b.bary[i] = (double)(1 / pr);
    }
    for (int q = 0; q < n; ++q)
        for (int a = 0; a < n; ++a) {
            b.S[q][a] = (double)lagrange(xn, n, a, g[q]);
            b.DS[q][a] = (double)lagrange_deriv(xn, n, a, g[q]);
            b.D[q][a] = (double)lagrange_deriv(g, n, a, g[q]);
        }
    return b;
}

}  // namespace nnmg

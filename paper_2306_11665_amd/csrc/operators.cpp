// Host construction of the 1D operators used by the kernels: nodes x and
// weights w of the Gauss-Legendre or Gauss-Lobatto rule on [-1, 1], the
// collocated Lagrange derivative D and Q = diag(w) D (the weighted 1D factor
// of Eq. (5)).  Built once per (n, node kind) in FP64 and cached.
//
// Gauss-Legendre nodes: Newton on P_n from Tricomi's asymptotic guesses, with
// P_n' from the recurrence P'_{k+1} = (k+1) P_k + x P'_k; weights
// w = 2 / ((1 - x)(1 + x) P_n'(x)^2).
// Gauss-Lobatto nodes: the roots of g = P_{N+1} - P_{N-1} (N = n - 1), which
// are +-1 and the roots of P_N'; Newton uses g' = (2N + 1) P_N.  Weights
// w = 2 / (N (N+1) P_N(x)^2).
// D: off-diagonal entries from the Lagrange product formula
// D_ij = prod_{k != i,j} (x_i - x_k) / prod_{k != j} (x_j - x_k); the
// diagonal is minus the off-diagonal row sum, so that D 1 = 0 to rounding
// (a constant state then gives a zero volume term).
#include "tensor_internal.h"

#include <cmath>
#include <mutex>
#include <vector>

namespace sfhad {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// P_k(x) for k = n and n - 1 via the three-term recurrence.
void legendre_pair(int n, double x, double &pn, double &pnm1) {
    double a = 1.0, b = x;  // P_0, P_1
    if (n == 0) { pn = 1.0; pnm1 = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double c = ((2 * k + 1) * x * b - k * a) / (k + 1);
        a = b;
        b = c;
    }
    pn = b;
    pnm1 = a;
}

// P_n(x) and P_n'(x), with P'_{k+1} = (k+1) P_k + x P'_k.
void legendre_with_derivative(int n, double x, double &p, double &dp) {
    double a = 1.0, b = x, db = 1.0;
    if (n == 0) { p = 1.0; dp = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double c = ((2 * k + 1) * x * b - k * a) / (k + 1);
        double dc = (k + 1) * b + x * db;
        a = b;
        b = c;
        db = dc;
    }
    p = b;
    dp = db;
}

double legendre_p(int n, double x) {
    double pn, pm;
    legendre_pair(n, x, pn, pm);
    return pn;
}

void gauss_legendre(int n, double *x, double *w) {
    for (int k = 1; k <= n; ++k) {
        // Tricomi: x_k ~ (1 - 1/(8n^2) + 1/(8n^3)) cos(pi (4k - 1) / (4n + 2)), descending in k
        double t = (1.0 - 1.0 / (8.0 * n * n) + 1.0 / (8.0 * n * n * n)) *
                   std::cos(kPi * (4.0 * k - 1.0) / (4.0 * n + 2.0));
        for (int it = 0; it < 60; ++it) {
            double pn, dp;
            legendre_with_derivative(n, t, pn, dp);
            double dt = pn / dp;
            t -= dt;
            if (std::fabs(dt) <= 1e-17) break;
        }
        double pn, dp;
        legendre_with_derivative(n, t, pn, dp);
        int i = n - k;  // ascending order
        x[i] = t;
        w[i] = 2.0 / ((1.0 - t) * (1.0 + t) * dp * dp);
    }
    if (n % 2 == 1) x[n / 2] = 0.0;  // the middle root is exactly zero
}

void gauss_lobatto(int n, double *x, double *w) {
    int N = n - 1;
    x[0] = -1.0;
    x[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double t = -std::cos(kPi * i / N);
        for (int it = 0; it < 60; ++it) {
            double g = legendre_p(N + 1, t) - legendre_p(N - 1, t);
            double dg = (2.0 * N + 1.0) * legendre_p(N, t);
            double dt = g / dg;
            t -= dt;
            if (std::fabs(dt) <= 1e-17) break;
        }
        x[i] = t;
    }
    if (n % 2 == 1) x[N / 2] = 0.0;
    for (int i = 0; i <= N; ++i) {
        double p = legendre_p(N, x[i]);
        w[i] = 2.0 / (N * (N + 1.0) * p * p);
    }
}

void derivative_matrix(int n, const double *x, double *D) {
    for (int j = 0; j < n; ++j) {
        double den = 1.0;
        for (int k = 0; k < n; ++k)
            if (k != j) den *= x[j] - x[k];
        for (int i = 0; i < n; ++i) {
            if (i == j) continue;
            double num = 1.0;
            for (int k = 0; k < n; ++k)
                if (k != i && k != j) num *= x[i] - x[k];
            D[i * n + j] = num / den;
        }
    }
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j)
            if (j != i) s += D[i * n + j];
        D[i * n + i] = -s;
    }
}

std::mutex g_mu;
std::vector<Operator1D> g_cache[2];  // index by node kind, then n

}  // namespace

bool build_operator(int n, int node_kind, Operator1D &op) {
    if (n < 1 || n > kMaxN) return false;
    if (node_kind != SF_NODES_GAUSS_LEGENDRE && node_kind != SF_NODES_GAUSS_LOBATTO) return false;
    if (node_kind == SF_NODES_GAUSS_LOBATTO && n < 2) return false;
    op.n = n;
    op.node_kind = node_kind;
    if (node_kind == SF_NODES_GAUSS_LEGENDRE)
        gauss_legendre(n, op.x, op.w);
    else
        gauss_lobatto(n, op.x, op.w);
    double D[kMaxN * kMaxN];
    derivative_matrix(n, op.x, D);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) op.Q[i * n + j] = op.w[i] * D[i * n + j];
    // Lagrange basis at x = -1 and +1, barycentric form
    // l_k(x) = (lambda_k / (x - x_k)) / sum_j lambda_j / (x - x_j); a node on the
    // end (Gauss-Lobatto) gives the unit vector exactly
    double lam[kMaxN];
    for (int j = 0; j < n; ++j) {
        double p = 1.0;
        for (int k = 0; k < n; ++k)
            if (k != j) p *= op.x[j] - op.x[k];
        lam[j] = 1.0 / p;
    }
    for (int side = 0; side < 2; ++side) {
        const double X = side ? 1.0 : -1.0;
        double *l = side ? op.lp : op.lm;
        int hit = -1;
        for (int k = 0; k < n; ++k)
            if (op.x[k] == X) hit = k;
        if (hit >= 0) {
            for (int k = 0; k < n; ++k) l[k] = k == hit ? 1.0 : 0.0;
            continue;
        }
        double den = 0.0;
        for (int j = 0; j < n; ++j) den += lam[j] / (X - op.x[j]);
        for (int k = 0; k < n; ++k) l[k] = (lam[k] / (X - op.x[k])) / den;
    }
    return true;
}

bool get_operator(int n, int node_kind, Operator1D &op) {
    if (node_kind != SF_NODES_GAUSS_LEGENDRE && node_kind != SF_NODES_GAUSS_LOBATTO) return false;
    std::lock_guard<std::mutex> lk(g_mu);
    auto &cache = g_cache[node_kind];
    if (cache.empty()) cache.resize(kMaxN + 1);
    if (n < 1 || n > kMaxN) return false;
    if (cache[n].n != n) {
        if (!build_operator(n, node_kind, cache[n])) return false;
    }
    op = cache[n];
    return true;
}

// Modal basis for the basis transformation: orthonormal Legendre
// polynomials L_k = sqrt((2k+1)/2) P_k evaluated on the n nodes,
// V[q][k] = L_k(x_q).  Its projection P = V^{-1} in closed form: the
// quadrature makes V^T W V = G diagonal -- the identity for Gauss-Legendre
// (exact to degree 2n - 1), and for Gauss-Lobatto the identity except
// G[N][N] = (2N + 1)/N (N = n - 1; the rule is exact to degree 2n - 3 and
// sums P_N^2 to 2/N) -- so P = G^{-1} V^T W.
bool build_basis(int n, int node_kind, double *V, double *P) {
    Operator1D op;
    if (!get_operator(n, node_kind, op)) return false;
    double Vl[kMaxN * kMaxN];
    for (int q = 0; q < n; ++q) {
        const double x = op.x[q];
        double pkm1 = 0.0, pk = 1.0;  // P_{-1}, P_0
        for (int k = 0; k < n; ++k) {
            Vl[q * n + k] = std::sqrt((2.0 * k + 1.0) / 2.0) * pk;
            const double pkp1 = ((2.0 * k + 1.0) * x * pk - k * pkm1) / (k + 1.0);
            pkm1 = pk;
            pk = pkp1;
        }
    }
    if (V)
        for (int i = 0; i < n * n; ++i) V[i] = Vl[i];
    if (P) {
        const int N = n - 1;
        for (int k = 0; k < n; ++k) {
            const double g = (node_kind == SF_NODES_GAUSS_LOBATTO && k == N) ? (2.0 * N + 1.0) / N : 1.0;
            for (int q = 0; q < n; ++q) P[k * n + q] = Vl[q * n + k] * op.w[q] / g;
        }
    }
    return true;
}

// n modes on m > n nodes: V[q][k] = L_k(x_q) (m x n); the m-point rule
// integrates the mass matrix exactly (degree 2n - 2 <= 2m - 3), so
// V^T W V = I and the L2 projection is P = V^T W (n x m).
bool build_basis_rect(int n, int m, int node_kind, double *V, double *P) {
    if (m == n) return build_basis(n, node_kind, V, P);
    if (m < n) return false;
    Operator1D op;
    if (!get_operator(m, node_kind, op)) return false;
    for (int q = 0; q < m; ++q) {
        const double x = op.x[q];
        double pkm1 = 0.0, pk = 1.0;
        for (int k = 0; k < n; ++k) {
            const double v = std::sqrt((2.0 * k + 1.0) / 2.0) * pk;
            if (V) V[q * n + k] = v;
            if (P) P[k * m + q] = v * op.w[q];
            const double pkp1 = ((2.0 * k + 1.0) * x * pk - k * pkm1) / (k + 1.0);
            pkm1 = pk;
            pk = pkp1;
        }
    }
    return true;
}

}  // namespace sfhad

// Host side of the prior-grid smoothing (Sec. 2.3.2, eq. smooth_grid): the
// eigendecomposition of the thin-plate penalty P of an n_E x n_x grid, which
// the finalize kernel uses to smooth the grid and to score GCV at any lambda.
//
// The penalty is the sum of squared finite-difference second derivatives,
// taken only where their stencils lie inside the grid:
//   (d2w/dE2)^2 at cells with a neighbour on both sides along E,
//   (d2w/dx2)^2 likewise along x, 2 (d2w/dEdx)^2 at interior cell corners.
// With S the (n-2) x n second-difference and F the (n-1) x n first-difference
// matrix of an axis of n cells of width h, A = S^T S / h^4 and B = F^T F / h^2,
//   P = A_E (x) I_x + 2 B_E (x) B_x + I_E (x) A_x   (cell k n_x + l).
// Every term is unchanged by reflecting an axis (k -> n-1-k), so P keeps the
// four subspaces of grids even or odd under the two reflections. In an
// orthonormal basis of even and odd vectors per axis, P splits into four
// blocks, each the same Kronecker sum of the axis operators projected onto one
// parity, and each is diagonalized alone: Householder reduction to tridiagonal
// form, then implicit symmetric QR steps with Wilkinson shifts, with the
// transformations accumulated (Golub & Van Loan, Matrix Computations,
// Sec. 8.3). A block of m cells costs about 9 m^3 flops instead of the
// 64 times larger cost of the whole grid.
//
// Layout of the basis (doubles): the eigenvalues of blocks 0..3, then the
// eigenvector matrices of blocks 0..3, each m_b x m_b row-major with entry
// [r][o] = component r of eigenvector o. Block b = 2 pE + pX (parity 0 even,
// 1 odd); its component (i, j) is at r = i m_X(pX) + j. Along an axis of n
// cells, even vector i < ceil(n/2) is (e_i + e_{n-1-i})/sqrt(2) (e_i alone at
// the middle cell of an odd n), odd vector i < floor(n/2) is
// (e_i - e_{n-1-i})/sqrt(2).
#include <cmath>
#include <cstddef>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "m2m_internal.h"

namespace m2m {
namespace {

// cells of parity p along an axis of n cells
int parity_count(int n, int p) { return p == 0 ? (n + 1) / 2 : n / 2; }

// the dense n x n axis operators: A = S^T S / h^4, B = F^T F / h^2
void axis_ops(int n, double h, std::vector<double>& A, std::vector<double>& B) {
    A.assign((size_t)n * n, 0.0);
    B.assign((size_t)n * n, 0.0);
    const double h2 = h * h, h4 = h2 * h2;
    for (int k = 1; k + 1 < n; ++k) {
        const int c[3] = {k - 1, k, k + 1};
        const double v[3] = {1.0, -2.0, 1.0};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) A[(size_t)c[a] * n + c[b]] += v[a] * v[b] / h4;
    }
    for (int k = 0; k + 1 < n; ++k) {
        const int c[2] = {k, k + 1};
        const double v[2] = {-1.0, 1.0};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) B[(size_t)c[a] * n + c[b]] += v[a] * v[b] / h2;
    }
}

// T^T M T for the n x m parity basis T of parity p (M dense n x n)
std::vector<double> project(const std::vector<double>& M, int n, int p) {
    const int m = parity_count(n, p);
    // column i of T: entries (k, coefficient)
    auto col = [n, p](int i, int* k, double* v) -> int {
        const int j = n - 1 - i;
        if (i == j) {
            k[0] = i;
            v[0] = 1.0;
            return 1;
        }
        const double s = std::sqrt(0.5);
        k[0] = i;
        v[0] = s;
        k[1] = j;
        v[1] = p == 0 ? s : -s;
        return 2;
    };
    std::vector<double> out((size_t)m * m, 0.0);
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            int ka[2], kb[2];
            double va[2], vb[2];
            const int na = col(a, ka, va), nb = col(b, kb, vb);
            double s = 0.0;
            for (int x = 0; x < na; ++x)
                for (int y = 0; y < nb; ++y) s += va[x] * M[(size_t)ka[x] * n + kb[y]] * vb[y];
            out[(size_t)a * m + b] = s;
        }
    return out;
}

// Householder reduction of the symmetric m x m matrix A (row-major, destroyed)
// to tridiagonal form: A = Q T Q^T with diagonal d and off-diagonal e
// (e[k] couples k and k+1); Q (m x m, row-major) is written.
void tridiagonalize(std::vector<double>& A, int m, std::vector<double>& d, std::vector<double>& e,
                    std::vector<double>& Q) {
    Q.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) Q[(size_t)i * m + i] = 1.0;
    std::vector<double> u(m), p(m), w(m), qu(m);
    for (int k = 0; k + 2 < m; ++k) {
        const int r = m - k - 1;  // length of the column below the diagonal
        double sig = 0.0;
        for (int t = 0; t < r; ++t) {
            const double x = A[(size_t)(k + 1 + t) * m + k];
            sig += x * x;
        }
        if (sig == 0.0) continue;
        const double x0 = A[(size_t)(k + 1) * m + k];
        const double alpha = x0 >= 0.0 ? -std::sqrt(sig) : std::sqrt(sig);
        // v = x - alpha e_1; H = I - u u^T with u = v sqrt(2 / v.v)
        double vv = 0.0;
        for (int t = 0; t < r; ++t) {
            u[t] = A[(size_t)(k + 1 + t) * m + k] - (t == 0 ? alpha : 0.0);
            vv += u[t] * u[t];
        }
        if (vv == 0.0) continue;
        const double sc = std::sqrt(2.0 / vv);
        for (int t = 0; t < r; ++t) u[t] *= sc;
        // trailing block S <- H S H = S - u w^T - w u^T, p = S u, w = p - (u.p / 2) u
        double up = 0.0;
        for (int a = 0; a < r; ++a) {
            double s = 0.0;
            const double* row = &A[(size_t)(k + 1 + a) * m + (k + 1)];
            for (int b = 0; b < r; ++b) s += row[b] * u[b];
            p[a] = s;
            up += u[a] * s;
        }
        for (int a = 0; a < r; ++a) w[a] = p[a] - 0.5 * up * u[a];
        for (int a = 0; a < r; ++a) {
            double* row = &A[(size_t)(k + 1 + a) * m + (k + 1)];
            for (int b = 0; b < r; ++b) row[b] -= u[a] * w[b] + w[a] * u[b];
        }
        A[(size_t)(k + 1) * m + k] = alpha;
        A[(size_t)k * m + (k + 1)] = alpha;
        for (int t = 1; t < r; ++t) {
            A[(size_t)(k + 1 + t) * m + k] = 0.0;
            A[(size_t)k * m + (k + 1 + t)] = 0.0;
        }
        // Q <- Q H on columns k+1..m-1
        for (int i = 0; i < m; ++i) {
            double* row = &Q[(size_t)i * m + (k + 1)];
            double s = 0.0;
            for (int t = 0; t < r; ++t) s += row[t] * u[t];
            for (int t = 0; t < r; ++t) row[t] -= s * u[t];
        }
    }
    d.resize(m);
    e.assign(m, 0.0);
    for (int i = 0; i < m; ++i) d[i] = A[(size_t)i * m + i];
    for (int i = 0; i + 1 < m; ++i) e[i] = A[(size_t)(i + 1) * m + i];
}

// Implicit symmetric QR steps with Wilkinson shifts on the tridiagonal (d, e)
// until every off-diagonal element is negligible; each Givens rotation G of
// rows/columns (k, k+1) maps T to G^T T G and Z to Z G. On return d holds the
// eigenvalues and the columns of Z the eigenvectors. False if it does not
// converge.
bool tridiagonal_qr(std::vector<double>& d, std::vector<double>& e, std::vector<double>& Z, int m) {
    const double eps = 2.220446049250313e-16;
    int hi = m - 1, iter = 0;
    while (hi > 0) {
        for (int i = 0; i < hi; ++i)
            if (std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1]))) e[i] = 0.0;
        if (e[hi - 1] == 0.0) {
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && e[lo - 1] != 0.0) --lo;
        if (++iter > 60 * m) return false;
        // shift: the eigenvalue of the trailing 2 x 2 closer to d[hi]
        const double dl = 0.5 * (d[hi - 1] - d[hi]);
        const double b = e[hi - 1];
        const double rt = std::hypot(dl, b);
        const double mu = d[hi] - b * b / (dl + (dl >= 0.0 ? rt : -rt));
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            // rotation that zeroes z against x (the bulge, or the shifted
            // first column at k = lo)
            const double r = std::hypot(x, z);
            const double c = x / r, s = -z / r;
            if (k > lo) e[k - 1] = r;
            const double dk = d[k], dk1 = d[k + 1], ek = e[k];
            d[k] = c * c * dk - 2.0 * c * s * ek + s * s * dk1;
            d[k + 1] = s * s * dk + 2.0 * c * s * ek + c * c * dk1;
            e[k] = c * s * (dk - dk1) + (c * c - s * s) * ek;
            if (k + 1 < hi) {
                z = -s * e[k + 1];
                e[k + 1] = c * e[k + 1];
                x = e[k];
            }
            for (int i = 0; i < m; ++i) {
                double* row = &Z[(size_t)i * m];
                const double a0 = row[k], a1 = row[k + 1];
                row[k] = c * a0 - s * a1;
                row[k + 1] = s * a0 + c * a1;
            }
        }
    }
    return true;
}

// eigenvalues g (m) and eigenvectors Z (m x m row-major, columns) of the
// symmetric matrix A
bool sym_eig(std::vector<double> A, int m, std::vector<double>& g, std::vector<double>& Z) {
    if (m == 0) {
        g.clear();
        Z.clear();
        return true;
    }
    std::vector<double> e;
    tridiagonalize(A, m, g, e, Z);
    return tridiagonal_qr(g, e, Z, m);
}

struct Basis {
    bool ok = false;
    std::vector<double> v;
};

using Key = std::tuple<int, int, double, double>;

std::mutex g_mu;
std::map<Key, std::shared_ptr<const Basis>> g_cache;

std::shared_ptr<const Basis> compute(int nE, int nx, double hE, double hx) {
    std::vector<double> AE, BE, AX, BX;
    axis_ops(nE, hE, AE, BE);
    axis_ops(nx, hx, AX, BX);
    std::vector<double> g[4], Z[4];
    bool ok[4] = {true, true, true, true};
    auto work = [&](int b) {
        const int pE = b >> 1, pX = b & 1;
        const int mE = parity_count(nE, pE), mX = parity_count(nx, pX), m = mE * mX;
        const std::vector<double> aE = project(AE, nE, pE), bE = project(BE, nE, pE);
        const std::vector<double> aX = project(AX, nx, pX), bX = project(BX, nx, pX);
        std::vector<double> M((size_t)m * m, 0.0);
        for (int i = 0; i < mE; ++i)
            for (int j = 0; j < mX; ++j)
                for (int i2 = 0; i2 < mE; ++i2)
                    for (int j2 = 0; j2 < mX; ++j2) {
                        double v = 2.0 * bE[(size_t)i * mE + i2] * bX[(size_t)j * mX + j2];
                        if (j == j2) v += aE[(size_t)i * mE + i2];
                        if (i == i2) v += aX[(size_t)j * mX + j2];
                        M[(size_t)(i * mX + j) * m + (i2 * mX + j2)] = v;
                    }
        ok[b] = sym_eig(std::move(M), m, g[b], Z[b]);
    };
    std::vector<std::thread> th;
    for (int b = 1; b < 4; ++b) th.emplace_back(work, b);
    work(0);
    for (auto& t : th) t.join();
    auto out = std::make_shared<Basis>();
    out->ok = ok[0] && ok[1] && ok[2] && ok[3];
    for (int b = 0; b < 4; ++b)
        for (double x : g[b]) out->v.push_back(x < 0.0 ? 0.0 : x);  // P is semidefinite
    for (int b = 0; b < 4; ++b) out->v.insert(out->v.end(), Z[b].begin(), Z[b].end());
    return out;
}

}  // namespace

size_t smooth_basis_len(int nE, int nx) {
    size_t len = (size_t)nE * nx;
    for (int b = 0; b < 4; ++b) {
        const size_t m = (size_t)parity_count(nE, b >> 1) * parity_count(nx, b & 1);
        len += m * m;
    }
    return len;
}

bool smooth_basis(int nE, int nx, double hE, double hx, double* out) {
    if (nE < 1 || nx < 1 || !(hE > 0) || !(hx > 0)) return false;
    const Key key{nE, nx, hE, hx};
    std::shared_ptr<const Basis> b;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) b = it->second;
    }
    if (!b) {
        b = compute(nE, nx, hE, hx);
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache.emplace(key, b);
    }
    if (!b->ok) return false;
    for (size_t i = 0; i < b->v.size(); ++i) out[i] = b->v[i];
    return true;
}

}  // namespace m2m

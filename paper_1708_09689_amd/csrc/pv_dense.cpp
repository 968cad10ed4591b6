// Small dense FP64 linear algebra on the host for the Rayleigh-Ritz steps of
// Chebyshev filter diagonalisation (Sec. 4.2): Cholesky factorisation,
// inversion of the triangular factor, and the cyclic Jacobi eigensolver for
// complex Hermitian matrices.  Matrices are row-major std::complex<double>,
// at most a few hundred rows (the search-space size), so O(n^3) host work is
// negligible next to the filter sweeps.
#include "pv_dense.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace pvd {

bool cholesky_upper(int n, std::vector<cd>& A) {
    // A = R^H R, R upper triangular; R overwrites the upper triangle of A,
    // the strict lower triangle is zeroed.
    for (int j = 0; j < n; ++j) {
        double d = A[(size_t)j * n + j].real();
        for (int k = 0; k < j; ++k) d -= std::norm(A[(size_t)k * n + j]);
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        const double rjj = std::sqrt(d);
        A[(size_t)j * n + j] = rjj;
        for (int i = j + 1; i < n; ++i) {
            cd s = A[(size_t)j * n + i];
            for (int k = 0; k < j; ++k) s -= std::conj(A[(size_t)k * n + j]) * A[(size_t)k * n + i];
            A[(size_t)j * n + i] = s / rjj;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) A[(size_t)i * n + j] = 0.0;
    return true;
}

void invert_upper(int n, const std::vector<cd>& R, std::vector<cd>& M) {
    // M = R^{-1} (upper triangular), by back substitution column by column.
    M.assign((size_t)n * n, cd(0.0));
    for (int j = 0; j < n; ++j) {
        M[(size_t)j * n + j] = 1.0 / R[(size_t)j * n + j];
        for (int i = j - 1; i >= 0; --i) {
            cd s = 0.0;
            for (int k = i + 1; k <= j; ++k) s += R[(size_t)i * n + k] * M[(size_t)k * n + j];
            M[(size_t)i * n + j] = -s / R[(size_t)i * n + i];
        }
    }
}

void heev_jacobi(int n, std::vector<cd>& A, std::vector<double>& w, std::vector<cd>& V) {
    // Cyclic Jacobi: each (p, q) rotation first removes the phase of A_pq
    // (diag(1, e^{-i phi})) and then applies the real symmetric Jacobi
    // rotation that zeroes |A_pq|.  V accumulates the product of rotations.
    V.assign((size_t)n * n, cd(0.0));
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    auto at = [&](int i, int j) -> cd& { return A[(size_t)i * n + j]; };
    for (int i = 0; i < n; ++i) at(i, i) = at(i, i).real();
    double scale = 0.0;
    for (const cd& v : A) scale = std::max(scale, std::abs(v));
    if (scale == 0.0) scale = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += std::norm(at(p, q));
        if (std::sqrt(off) <= 1e-17 * scale * n) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const cd apq = at(p, q);
                const double r = std::abs(apq);
                if (r <= 1e-300 || r < 1e-18 * scale) continue;
                const cd e = apq / r;                    // e^{i phi}
                const double a = at(p, p).real(), b = at(q, q).real();
                const double theta = (b - a) / (2.0 * r);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                const cd ec = std::conj(e);
                // U = [[cs, sn], [-sn e^{-i phi}, cs e^{-i phi}]] on (p, q)
                const cd upp = cs, upq = sn, uqp = -sn * ec, uqq = cs * ec;
                for (int k = 0; k < n; ++k) {  // A <- A U (columns p, q)
                    const cd akp = at(k, p), akq = at(k, q);
                    at(k, p) = akp * upp + akq * uqp;
                    at(k, q) = akp * upq + akq * uqq;
                }
                for (int k = 0; k < n; ++k) {  // A <- U^H A (rows p, q)
                    const cd apk = at(p, k), aqk = at(q, k);
                    at(p, k) = std::conj(upp) * apk + std::conj(uqp) * aqk;
                    at(q, k) = std::conj(upq) * apk + std::conj(uqq) * aqk;
                }
                at(p, q) = 0.0;
                at(q, p) = 0.0;
                at(p, p) = at(p, p).real();
                at(q, q) = at(q, q).real();
                for (int k = 0; k < n; ++k) {  // V <- V U
                    const cd vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = vkp * upp + vkq * uqp;
                    V[(size_t)k * n + q] = vkp * upq + vkq * uqq;
                }
            }
    }
    // ascending eigenvalues, columns of V permuted alike
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int i, int j) { return at(i, i).real() < at(j, j).real(); });
    w.resize(n);
    std::vector<cd> Vs((size_t)n * n);
    for (int c = 0; c < n; ++c) {
        w[c] = at(idx[c], idx[c]).real();
        for (int k = 0; k < n; ++k) Vs[(size_t)k * n + c] = V[(size_t)k * n + idx[c]];
    }
    V.swap(Vs);
}

}  // namespace pvd

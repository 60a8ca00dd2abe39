// Host-side checks of the library's precomputation routines (tvd_plan.cpp)
// against facts of the mathematics, built with g++ and the address /
// undefined-behaviour sanitizers by tests/test_host_plan.py.  Prints one
// line per check and exits non-zero on the first failure.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "tvd_internal.hpp"

namespace {

int failures = 0;

void check(bool ok, const char* what, double err) {
    std::printf("%-60s %s (%.3g)\n", what, ok ? "ok" : "FAIL", err);
    if (!ok) ++failures;
}

std::vector<double> matmul(const std::vector<double>& A, const std::vector<double>& B, int n) {
    std::vector<double> C(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j) C[size_t(i) * n + j] += A[size_t(i) * n + k] * B[size_t(k) * n + j];
    return C;
}

// symmetric normalised 1D filter of half-width m
std::vector<double> filter(int m, unsigned seed) {
    std::vector<double> g(2 * m + 1);
    double sum = 0.0;
    for (int a = 0; a <= m; ++a) {
        seed = seed * 1103515245u + 12345u;
        const double q = 0.05 + double(seed % 1000) / 1000.0;
        g[m + a] = g[m - a] = q;
    }
    for (double x : g) sum += x;
    for (double& x : g) x /= sum;
    return g;
}

}  // namespace

int main() {
    const double eps = 2.220446049250313e-16;
    // T_n^{-1} T_n = I (Section 2's closed-form inverse)
    for (int n : {3, 4, 5, 7, 64, 130}) {
        std::vector<double> T, Ti;
        tvd::ar_transform_matrices(n, T, Ti);
        const std::vector<double> P = matmul(Ti, T, n);
        double e = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) e = std::fmax(e, std::fabs(P[size_t(i) * n + j] - (i == j ? 1.0 : 0.0)));
        char what[96];
        std::snprintf(what, sizeof what, "T_n^{-1} T_n = I, n = %d", n);
        check(e < 64 * n * eps, what, e);
    }
    // end weights: sum 1 (AR(I) = I), absolute sum n - 2 (alternating extrapolation)
    for (int n : {3, 5, 40, 130, 512}) {
        const std::vector<double> w = tvd::ar_end_weights(n);
        double s = 0.0, sa = 0.0;
        for (double x : w) {
            s += x;
            sa += std::fabs(x);
        }
        char what[96];
        std::snprintf(what, sizeof what, "end weights: sum 1, absolute sum n - 2, n = %d", n);
        const double e = std::fmax(std::fabs(s - 1.0), std::fabs(sa - (n - 2)) / n);
        check(int(w.size()) == n - 2 && e < 1e-9, what, e);
        // closed form: w_j = (-1)^(j+1) (1 + cos(j pi / (n - 1))), j = 1..n-2
        double ec = 0.0;
        for (int j = 1; j <= n - 2; ++j) {
            const double c = ((j & 1) ? 1.0 : -1.0) * (1.0 + std::cos(3.14159265358979323846 * j / (n - 1)));
            ec = std::fmax(ec, std::fabs(w[j - 1] - c));
        }
        std::snprintf(what, sizeof what, "end weights = (-1)^(j+1) (1 + cos theta_j), n = %d", n);
        check(ec < 2.0 * n * n * eps, what, ec);
    }
    // T_n^{-1} H T_n = diag(symbol on the y = 0 grid) for anti-reflective blurs (Section 2)
    for (int n : {7, 12, 33}) {
        for (int m : {1, 2, 3}) {
            const std::vector<double> g = filter(m, unsigned(7 * n + m));
            const std::vector<double> H = tvd::blur_matrix_1d(g, n, 2);
            std::vector<double> T, Ti;
            tvd::ar_transform_matrices(n, T, Ti);
            const std::vector<double> D = matmul(matmul(Ti, H, n), T, n);
            double off = 0.0, diag = 0.0;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    if (i != j) {
                        off = std::fmax(off, std::fabs(D[size_t(i) * n + j]));
                        continue;
                    }
                    // grid: y_0 = 0, y_i = i pi / (n - 1) for 0 < i < n - 1, y_{n-1} = 0
                    const double y = (i == n - 1) ? 0.0 : 3.14159265358979323846 * i / (n - 1);
                    double sym = 0.0;
                    for (int a = -m; a <= m; ++a) sym += g[a + m] * std::cos(a * y);
                    diag = std::fmax(diag, std::fabs(D[size_t(i) * n + i] - sym));
                }
            char what[96];
            std::snprintf(what, sizeof what, "T^{-1} H T diagonal with the symbol, n = %d, m = %d", n, m);
            check(off < 1e3 * n * eps && diag < 1e3 * n * eps, what, std::fmax(off, diag));
        }
    }
    // H H is banded with half-width 2m: its band holds the whole product, and
    // the Toeplitz-compressed band reproduces every row
    for (int n : {9, 20, 45}) {
        const int m = 3;
        const std::vector<double> g = filter(m, unsigned(n));
        const std::vector<double> H = tvd::blur_matrix_1d(g, n, 2);
        const std::vector<double> HH = tvd::matmul_tn(tvd::transpose(H, n), H, n);
        const std::vector<double> ref = matmul(H, H, n);
        const int w = 2 * m, bw = 2 * w + 1;
        const std::vector<double> band = tvd::band_of(HH, n, w);
        double e = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const int d = j - i;
                const double b = (d >= -w && d <= w) ? band[size_t(i) * bw + d + w] : 0.0;
                e = std::fmax(e, std::fabs(b - ref[size_t(i) * n + j]));
            }
        const tvd::ToeplitzBand tb = tvd::compress_band(band, n, w);
        double ec = 0.0;
        for (int i = 0; i < n; ++i) {
            const int rr = i < tb.lo ? 1 + i : (i >= tb.hi ? 1 + tb.lo + (i - tb.hi) : 0);
            for (int d = 0; d < bw; ++d)
                ec = std::fmax(ec, std::fabs(tb.data[size_t(rr) * bw + d] - band[size_t(i) * bw + d]));
        }
        char what[96];
        std::snprintf(what, sizeof what, "H H band and its compressed rows, n = %d", n);
        check(e < 64 * eps && ec == 0.0, what, std::fmax(e, ec));
    }
    // periodic (bc 4): the real Fourier basis is orthonormal and diagonalises
    // the circulant blur with the symbol at 2 pi f / n; zero-Dirichlet (bc 3):
    // the eigenvalues equal diag(P^T H P) over the DCT-II basis
    for (int n : {5, 8, 13, 16}) {
        for (int m : {1, 2}) {
            const std::vector<double> g = filter(m, unsigned(11 * n + m));
            std::vector<double> h2(g.size());  // 1 x (2m+1) PSF
            for (size_t i = 0; i < g.size(); ++i) h2[i] = g[i];
            for (int bc : {3, 4}) {
                const std::vector<double> H = tvd::blur_matrix_1d(g, n, bc);
                const std::vector<double> P = tvd::basis_matrix(n, bc);  // P[i*n+k] = phi_k(i)
                const std::vector<double> D = matmul(matmul(tvd::transpose(P, n), H, n), P, n);
                const std::vector<double> O = matmul(tvd::transpose(P, n), P, n);
                const std::vector<double> lam = tvd::symbol_eigenvalues(h2.data(), 1, 2 * m + 1, 3, n, bc);
                double off = 0.0, diag = 0.0, orth = 0.0;
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) {
                        orth = std::fmax(orth, std::fabs(O[size_t(i) * n + j] - (i == j ? 1.0 : 0.0)));
                        if (i == j) diag = std::fmax(diag, std::fabs(D[size_t(i) * n + i] - lam[i]));
                        else off = std::fmax(off, std::fabs(D[size_t(i) * n + j]));
                    }
                char what[96];
                std::snprintf(what, sizeof what, "%s basis and eigenvalues, n = %d, m = %d",
                              bc == 4 ? "periodic" : "zero-Dirichlet", n, m);
                const bool ok = orth < 64 * n * eps && diag < 1e3 * n * eps && (bc == 3 || off < 1e3 * n * eps);
                check(ok, what, std::fmax(orth, std::fmax(diag, bc == 4 ? off : 0.0)));
            }
        }
    }
    std::printf("%s\n", failures ? "FAILED" : "all ok");
    return failures ? 1 : 0;
}

// Host-side precomputation for libtvdeblur (FP64): PSF validation and
// factorisation, 1D blur matrices with the boundary condition folded in,
// bands for the device operators, transform tables, basis matrices and the
// PSF symbol on each boundary condition's grid.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>

#include "tvd_internal.hpp"

namespace tvd {

namespace {
const double kPi = 3.14159265358979323846264338327950288;

// cos / sin of pi * num / den with exact integer range reduction.
double cos_pi_frac(long long num, long long den) {
    long long r = num % (2 * den);
    if (r < 0) r += 2 * den;
    return std::cos(kPi * double(r) / double(den));
}
double sin_pi_frac(long long num, long long den) {
    long long r = num % (2 * den);
    if (r < 0) r += 2 * den;
    return std::sin(kPi * double(r) / double(den));
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

void fft_host(std::vector<std::complex<double>>& a) {  // iterative radix-2, forward
    const size_t n = a.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        for (size_t i = 0; i < n; i += len) {
            for (size_t k = 0; k < len / 2; ++k) {
                // twiddle exp(-2 pi i k / len) with exact reduction
                const double c = cos_pi_frac(2LL * k, (long long)len);
                const double s = -sin_pi_frac(2LL * k, (long long)len);
                const std::complex<double> w(c, s);
                const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w;
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
        }
    }
}

// One-sided Jacobi SVD of a (rows x cols) row-major matrix, rows >= cols.
// Returns singular values and left/right singular vectors.
void jacobi_svd(std::vector<double> A, int rows, int cols, std::vector<double>& sig,
                std::vector<std::vector<double>>& U, std::vector<std::vector<double>>& V) {
    std::vector<double> Vm(size_t(cols) * cols, 0.0);
    for (int i = 0; i < cols; ++i) Vm[size_t(i) * cols + i] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < cols; ++p)
            for (int q = p + 1; q < cols; ++q) {
                double al = 0, be = 0, ga = 0;
                for (int i = 0; i < rows; ++i) {
                    const double ap = A[size_t(i) * cols + p], aq = A[size_t(i) * cols + q];
                    al += ap * ap;
                    be += aq * aq;
                    ga += ap * aq;
                }
                if (ga == 0.0 || std::fabs(ga) <= 1e-17 * std::sqrt(al * be)) continue;
                off = std::max(off, std::fabs(ga) / std::sqrt(al * be));
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
                for (int i = 0; i < rows; ++i) {
                    const double ap = A[size_t(i) * cols + p], aq = A[size_t(i) * cols + q];
                    A[size_t(i) * cols + p] = c * ap - s * aq;
                    A[size_t(i) * cols + q] = s * ap + c * aq;
                }
                for (int i = 0; i < cols; ++i) {
                    const double vp = Vm[size_t(i) * cols + p], vq = Vm[size_t(i) * cols + q];
                    Vm[size_t(i) * cols + p] = c * vp - s * vq;
                    Vm[size_t(i) * cols + q] = s * vp + c * vq;
                }
            }
        if (off < 1e-16) break;
    }
    sig.assign(cols, 0.0);
    U.assign(cols, std::vector<double>(rows, 0.0));
    V.assign(cols, std::vector<double>(cols, 0.0));
    for (int j = 0; j < cols; ++j) {
        double nrm = 0;
        for (int i = 0; i < rows; ++i) nrm += A[size_t(i) * cols + j] * A[size_t(i) * cols + j];
        nrm = std::sqrt(nrm);
        sig[j] = nrm;
        for (int i = 0; i < rows; ++i) U[j][i] = nrm > 0 ? A[size_t(i) * cols + j] / nrm : 0.0;
        for (int i = 0; i < cols; ++i) V[j][i] = Vm[size_t(i) * cols + j];
    }
}
}  // namespace

int validate_psf(const double* h, int py, int px, std::string& err) {
    if (!h || py < 1 || px < 1 || py % 2 == 0 || px % 2 == 0) {
        err = "PSF sizes must be positive and odd";
        return -1;
    }
    const int my = py / 2, mx = px / 2;
    double mx_abs = 0, sum = 0;
    for (int k = 0; k < py * px; ++k) {
        if (!std::isfinite(h[k])) {
            err = "PSF has a non-finite entry";
            return -1;
        }
        mx_abs = std::max(mx_abs, std::fabs(h[k]));
        sum += h[k];
    }
    const double tol = 1e-12 * mx_abs;
    for (int a = -my; a <= my; ++a)
        for (int b = -mx; b <= mx; ++b) {
            const double v = h[(a + my) * px + b + mx];
            if (std::fabs(v - h[(-a + my) * px + b + mx]) > tol || std::fabs(v - h[(a + my) * px - b + mx]) > tol) {
                err = "PSF is not quadrantally symmetric";
                return -2;
            }
        }
    if (std::fabs(sum - 1.0) > 1e-12) {
        err = "PSF does not sum to 1";
        return -3;
    }
    return 0;
}

PsfFactors factor_psf(const double* h, int py, int px) {
    PsfFactors f;
    f.my = py / 2;
    f.mx = px / 2;
    double mabs = 0;
    for (int k = 0; k < py * px; ++k) mabs = std::max(mabs, std::fabs(h[k]));
    // rank-1 test through the centre row and column
    const double c = h[f.my * px + f.mx];
    if (c > 0) {
        double err = 0;
        for (int a = 0; a < py; ++a)
            for (int b = 0; b < px; ++b)
                err = std::max(err, std::fabs(h[a * px + b] - h[a * px + f.mx] * h[f.my * px + b] / c));
        if (err <= 1e-14 * mabs) {
            std::vector<double> gy(py), gx(px);
            const double sc = std::sqrt(c);
            for (int a = 0; a < py; ++a) gy[a] = h[a * px + f.mx] / sc;
            for (int b = 0; b < px; ++b) gx[b] = h[f.my * px + b] / sc;
            f.gy.push_back(gy);
            f.gx.push_back(gx);
            f.rank = 1;
            return f;
        }
    }
    // general: SVD truncated at the numerical rank
    const bool tr = py < px;
    const int rows = tr ? px : py, cols = tr ? py : px;
    std::vector<double> A(size_t(rows) * cols);
    for (int a = 0; a < py; ++a)
        for (int b = 0; b < px; ++b) {
            if (tr) A[size_t(b) * cols + a] = h[a * px + b];
            else A[size_t(a) * cols + b] = h[a * px + b];
        }
    std::vector<double> sig;
    std::vector<std::vector<double>> U, V;
    jacobi_svd(A, rows, cols, sig, U, V);
    std::vector<int> order(cols);
    for (int j = 0; j < cols; ++j) order[j] = j;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return sig[x] > sig[y]; });
    const double smax = sig[order[0]];
    for (int jj = 0; jj < cols; ++jj) {
        const int j = order[jj];
        if (sig[j] <= 1e-15 * smax) break;
        std::vector<double> left = U[j], right = V[j];  // A = sum sig u v^T
        for (double& v : left) v *= sig[j];
        if (tr) {
            f.gy.push_back(right);
            f.gx.push_back(left);
        } else {
            f.gy.push_back(left);
            f.gx.push_back(right);
        }
    }
    f.rank = int(f.gy.size());
    return f;
}

std::vector<double> blur_matrix_1d(const std::vector<double>& g, int n, int bc) {
    const int m = int(g.size()) / 2;
    std::vector<double> H(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int a = -m; a <= m; ++a) {
            const double w = g[a + m];
            const int e = i - a;  // (H u)_i = sum_a g_a u~_{i-a}
            double* row = &H[size_t(i) * n];
            if (e >= 0 && e < n) {
                row[e] += w;
            } else if (bc == 3) {  // zero ghosts: Toeplitz
                continue;
            } else if (bc == 4) {  // periodic ghosts: circulant (m <= n)
                row[(e % n + n) % n] += w;
            } else if (e < 0) {
                const int j = -e;
                if (bc == 2) {  // u~_{-j} = 2u_0 - u_j
                    row[0] += 2 * w;
                    row[j] -= w;
                } else {        // u~_{-j} = u_{j-1}
                    row[j - 1] += w;
                }
            } else {
                const int j = e - (n - 1);
                if (bc == 2) {  // u~_{n-1+j} = 2u_{n-1} - u_{n-1-j}
                    row[n - 1] += 2 * w;
                    row[n - 1 - j] -= w;
                } else {        // u~_{n-1+j} = u_{n-j}
                    row[n - j] += w;
                }
            }
        }
    return H;
}

std::vector<double> band_wrapped(const std::vector<double>& A, int n, int w) {
    const int bw = 2 * w + 1;
    std::vector<double> out(size_t(n) * bw, 0.0);
    for (int i = 0; i < n; ++i)
        for (int d = -w; d <= w; ++d) out[size_t(i) * bw + d + w] = A[size_t(i) * n + ((i + d) % n + n) % n];
    return out;
}

std::vector<double> band_of(const std::vector<double>& A, int n, int w) {
    const int bw = 2 * w + 1;
    std::vector<double> out(size_t(n) * bw, 0.0);
    for (int i = 0; i < n; ++i)
        for (int d = -w; d <= w; ++d) {
            const int j = i + d;
            if (j >= 0 && j < n) out[size_t(i) * bw + d + w] = A[size_t(i) * n + j];
        }
    return out;
}

ToeplitzBand compress_band(const std::vector<double>& band, int n, int w) {
    const int bw = 2 * w + 1;
    ToeplitzBand t;
    t.w = w;
    const int mid = n / 2;
    auto same = [&](int i) {
        for (int d = 0; d < bw; ++d)
            if (band[size_t(i) * bw + d] != band[size_t(mid) * bw + d]) return false;
        return true;
    };
    int lo = mid, hi = mid + 1;
    while (lo > 0 && same(lo - 1)) --lo;
    while (hi < n && same(hi)) ++hi;
    // Equality includes the zero taps that fall outside the image, so using
    // the Toeplitz row for every row in [lo, hi) is exact.
    t.lo = lo;
    t.hi = hi;
    t.data.assign(band.begin() + size_t(mid) * bw, band.begin() + size_t(mid + 1) * bw);
    t.data.insert(t.data.end(), band.begin(), band.begin() + size_t(lo) * bw);
    t.data.insert(t.data.end(), band.begin() + size_t(hi) * bw, band.end());
    return t;
}

std::vector<double> transpose(const std::vector<double>& A, int n) {
    std::vector<double> T(size_t(n) * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) T[size_t(j) * n + i] = A[size_t(i) * n + j];
    return T;
}

std::vector<double> matmul_tn(const std::vector<double>& A, const std::vector<double>& B, int n) {
    // C = A^T B for banded-ish dense n x n (A, B of bandwidth << n are cheap
    // because zero rows are skipped).
    std::vector<double> C(size_t(n) * n, 0.0);
    for (int t = 0; t < n; ++t) {
        const double* a = &A[size_t(t) * n];
        const double* b = &B[size_t(t) * n];
        int lo = n, hi = -1, lob = n, hib = -1;
        for (int k = 0; k < n; ++k) {
            if (a[k] != 0.0) { lo = std::min(lo, k); hi = std::max(hi, k); }
            if (b[k] != 0.0) { lob = std::min(lob, k); hib = std::max(hib, k); }
        }
        for (int i = lo; i <= hi; ++i) {
            if (a[i] == 0.0) continue;
            double* c = &C[size_t(i) * n];
            for (int j = lob; j <= hib; ++j) c[j] += a[i] * b[j];
        }
    }
    return C;
}

// T_n of the anti-reflective algebra (Section 2): columns (1, p, 0),
// (0, S_{n-2}, 0), (0, Jp, 1) with p_j = 1 - j/(n-1), j = 1..n-2; and its
// inverse with interior rows (-S p, S, -S J p).
void ar_transform_matrices(int n, std::vector<double>& T, std::vector<double>& Ti) {
    const int m = n - 2;
    const double sc = std::sqrt(2.0 / (m + 1));
    std::vector<double> S(size_t(m) * m), p(m), sp(m, 0.0), sjp(m, 0.0);
    for (int i = 0; i < m; ++i) {
        p[i] = 1.0 - double(i + 1) / double(n - 1);
        for (int j = 0; j < m; ++j) S[size_t(i) * m + j] = sc * sin_pi_frac((long long)(i + 1) * (j + 1), m + 1);
    }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            sp[i] += S[size_t(i) * m + j] * p[j];
            sjp[i] += S[size_t(i) * m + j] * p[m - 1 - j];
        }
    T.assign(size_t(n) * n, 0.0);
    Ti.assign(size_t(n) * n, 0.0);
    T[0] = Ti[0] = 1.0;
    T[size_t(n) * n - 1] = Ti[size_t(n) * n - 1] = 1.0;
    for (int i = 1; i <= m; ++i) {
        double* t = &T[size_t(i) * n];
        double* ti = &Ti[size_t(i) * n];
        t[0] = p[i - 1];
        t[n - 1] = p[m - i];
        ti[0] = -sp[i - 1];
        ti[n - 1] = -sjp[i - 1];
        for (int j = 1; j <= m; ++j) t[j] = ti[j] = S[size_t(i - 1) * m + j - 1];
    }
}

// End eigenvalue of AR(A) (Section 3): the corner entry z_1 + 2 sum_{k>=2} z_k,
// with z the generator of the tau matrix s(A_in) = S diag(mu) S, is linear in
// mu.  For mu = e_j the first column of S diag(e_j) S is c_k = S_kj S_1j, and
// c_k = z_k - z_{k+2} gives z from the last entry up.
std::vector<double> ar_end_weights(int n) {
    const int m = n - 2;
    const double sc = std::sqrt(2.0 / (m + 1));
    std::vector<double> w(m), z(m + 2);
    for (int j = 0; j < m; ++j) {
        const double s1 = sc * sin_pi_frac(j + 1, m + 1);
        z[m] = z[m + 1] = 0.0;
        for (int k = m - 1; k >= 0; --k) z[k] = sc * sin_pi_frac((long long)(k + 1) * (j + 1), m + 1) * s1 + z[k + 2];
        double acc = 0.0;
        for (int k = 1; k < m; ++k) acc += z[k];
        w[j] = z[0] + 2.0 * acc;
    }
    return w;
}

std::vector<double> basis_matrix(int n, int bc) {
    std::vector<double> P(size_t(n) * n, 0.0);
    if (bc == 4) {  // real Fourier: 1, cos/sin pairs of frequency f, (-1)^i for even n
        for (int i = 0; i < n; ++i) {
            P[size_t(i) * n] = 1.0 / std::sqrt(double(n));
            for (int k = 1; k < n; ++k) {
                const int f = (k + 1) / 2;
                double v;
                if (n % 2 == 0 && k == n - 1) v = ((i & 1) ? -1.0 : 1.0) / std::sqrt(double(n));
                else if (k & 1) v = std::sqrt(2.0 / n) * cos_pi_frac(2LL * f * i, n);
                else v = std::sqrt(2.0 / n) * sin_pi_frac(2LL * f * i, n);
                P[size_t(i) * n + k] = v;
            }
        }
        return P;
    }
    if (bc == 1 || bc == 3) {  // DCT-II: phi_k(i) = sqrt((2 - [k=0])/n) cos(pi k (2i+1) / (2n))
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k)
                P[size_t(i) * n + k] =
                    std::sqrt((k == 0 ? 1.0 : 2.0) / n) * cos_pi_frac((long long)k * (2 * i + 1), 2LL * n);
    } else {        // S^ = diag(1, S_{n-2}, 1)
        P[0] = 1.0;
        P[size_t(n - 1) * n + n - 1] = 1.0;
        const double sc = std::sqrt(2.0 / (n - 1));
        for (int i = 1; i < n - 1; ++i)
            for (int k = 1; k < n - 1; ++k) P[size_t(i) * n + k] = sc * sin_pi_frac((long long)i * k, n - 1);
    }
    return P;
}

std::vector<double> symbol_eigenvalues(const double* h, int py, int px, int ny, int nx, int bc) {
    const int my = py / 2, mx = px / 2;
    // theta_k = pi num_k / den
    auto grid = [&](int n, std::vector<long long>& num, long long& den) {
        num.assign(n, 0);
        if (bc == 1) {
            den = n;
            for (int k = 0; k < n; ++k) num[k] = k;
        } else if (bc == 4) {  // 2 pi f / n for the cosine and sine rows of frequency f
            den = n;
            for (int k = 1; k < n; ++k) num[k] = 2LL * ((k + 1) / 2);
        } else {
            den = n - 1;
            for (int k = 1; k < n - 1; ++k) num[k] = k;
        }
    };
    // lam = Cy h Cx^T with C[k][a] = cos(a theta_k) on the BC grid, or for
    // zero-Dirichlet BCs (Toeplitz blur) C[k][a] = sum_i phi_k(i) phi_k(i+a)
    // over the DCT-II basis: the optimal cosine-algebra projection
    // diag(Q2 H Q2^T), the blur being sum_ab h_ab Z_a (x) Z_b with zero-fill
    // shifts Z_a.
    auto table = [&](int n, int m, std::vector<double>& C) {
        const int w = 2 * m + 1;
        C.assign(size_t(n) * w, 0.0);
        if (bc == 3) {
            const std::vector<double> P = basis_matrix(n, 3);  // P[i*n + k] = phi_k(i)
            for (int k = 0; k < n; ++k)
                for (int a = -m; a <= m; ++a) {
                    double s = 0.0;
                    const int lo = std::max(0, -a), hi = std::min(n, n - a);
                    for (int i = lo; i < hi; ++i) s += P[size_t(i) * n + k] * P[size_t(i + a) * n + k];
                    C[size_t(k) * w + a + m] = s;
                }
            return;
        }
        std::vector<long long> num;
        long long den;
        grid(n, num, den);
        for (int k = 0; k < n; ++k)
            for (int a = -m; a <= m; ++a) C[size_t(k) * w + a + m] = cos_pi_frac(a * num[k], den);
    };
    std::vector<double> Cy, Cx;
    table(ny, my, Cy);
    table(nx, mx, Cx);
    std::vector<double> tmp(size_t(ny) * px, 0.0);  // Cy h
    for (int k = 0; k < ny; ++k)
        for (int a = 0; a < py; ++a) {
            const double c = Cy[size_t(k) * py + a];
            for (int b = 0; b < px; ++b) tmp[size_t(k) * px + b] += c * h[a * px + b];
        }
    std::vector<double> lam(size_t(ny) * nx, 0.0);
    for (int k = 0; k < ny; ++k)
        for (int l = 0; l < nx; ++l) {
            double s = 0;
            for (int b = 0; b < px; ++b) s += tmp[size_t(k) * px + b] * Cx[size_t(l) * px + b];
            lam[size_t(k) * nx + l] = s;
        }
    return lam;
}

AxisTables make_axis_tables(int n, int bc) {
    AxisTables t;
    t.n = n;
    t.kind = (bc == 2) ? 1 : 2;  // zero-Dirichlet uses the reflective DCT-II
    t.L = (t.kind == 1) ? 2 * (n - 1) : 2 * n;
    if (is_pow2(t.L)) {
        t.M = t.L;
        t.bluestein = 0;
    } else {
        t.M = 1;
        while (t.M < 2 * t.L - 1) t.M <<= 1;
        t.bluestein = 1;
    }
    t.log2M = 0;
    while ((1 << t.log2M) < t.M) ++t.log2M;
    t.tw.resize(2 * size_t(t.M));  // M complex
    for (int k = 0; k < t.M; ++k) {
        t.tw[2 * k] = cos_pi_frac(2LL * k, t.M);
        t.tw[2 * k + 1] = -sin_pi_frac(2LL * k, t.M);
    }
    if (t.bluestein) {
        const long long L = t.L;
        t.chirp.resize(2 * size_t(L));
        std::vector<std::complex<double>> b(t.M, 0.0);
        for (long long k = 0; k < L; ++k) {
            const long long r = (k * k) % (2 * L);  // exp(-i pi k^2 / L)
            const double c = cos_pi_frac(r, L), s = -sin_pi_frac(r, L);
            t.chirp[2 * k] = c;
            t.chirp[2 * k + 1] = s;
            b[k] = std::complex<double>(c, -s);
            if (k > 0) b[t.M - k] = std::complex<double>(c, -s);
        }
        fft_host(b);
        t.bf.resize(2 * size_t(t.M));
        for (int k = 0; k < t.M; ++k) {
            t.bf[2 * k] = b[k].real() / t.M;
            t.bf[2 * k + 1] = b[k].imag() / t.M;
        }
    }
    if (t.kind == 2) {
        t.pre.resize(2 * size_t(n));
        t.post.resize(2 * size_t(n));
        for (int k = 0; k < n; ++k) {
            const double w = std::sqrt((k == 0 ? 1.0 : 2.0) / n);
            const double c = cos_pi_frac(k, 2LL * n), s = sin_pi_frac(k, 2LL * n);
            t.pre[2 * k] = w * c;
            t.pre[2 * k + 1] = w * s;
            t.post[2 * k] = 0.5 * w * c;
            t.post[2 * k + 1] = -0.5 * w * s;
        }
    }
    t.dst_scale = 1.0 / std::sqrt(2.0 * (n - 1));
    // one blob: every section padded to an even number of complex entries
    auto add = [&](const std::vector<double>& v) {
        const int off = int(t.blob.size() / 2);
        t.blob.insert(t.blob.end(), v.begin(), v.end());
        if ((v.size() / 2) % 2) t.blob.insert(t.blob.end(), {0.0, 0.0});
        return off;
    };
    add(t.tw);
    t.off_chirp = add(t.chirp);
    t.off_bf = add(t.bf);
    t.off_pre = add(t.pre);
    t.off_post = add(t.post);
    t.blob_len = int(t.blob.size() / 2);
    return t;
}

}  // namespace tvd

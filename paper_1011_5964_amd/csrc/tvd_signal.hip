// 1D signal deblurring (Section 5.1): many independent signals, one launch.
//
// Each signal is its own instance of the lagged-diffusivity method of eq. (fp)
// in one dimension -- (H^T H + alpha L(u^k)) u^{k+1} = H^T v, u^0 = v, PCG
// warm-started at u^k with the preconditioners of Section 3 (I, D of eq. (D),
// X = R or M, D_X, X_D) -- and runs entirely inside one workgroup: the
// fixed-point loop, every PCG iteration, the per-step eigenvalue setup and the
// stopping tests, with the workgroup barrier as the only synchronisation.  A
// batch of signals (the alpha / beta / preconditioner sweeps of Tables 1-2,
// the n sweep of the paper's iteration-count figure) is one kernel launch with
// no host round trip.  All arithmetic is IEEE double, the paper's precision.
//
// Layout per signal (device, FP64): the band of H^T H (n x (4m+1), the BC
// folded into its coefficients), the band of H^T (n x (2m+1)), the basis
// matrix Phi[i*n + k] = phi_k(i) of the BC's transform and its transpose,
// lambda_H^2 on the BC grid, and a work area of 11 n doubles.  The transforms
// are dense matrix-vector products with Phi: at these lengths (n in the
// hundreds to a few thousand) a workgroup streams Phi from L2 faster than it
// would run a mixed-radix FFT of the awkward lengths 2(n-1).

#include "../../include/tvdeblur.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "tvd_internal.hpp"

namespace tvd {
namespace {

constexpr int kSigThreads = 256;
constexpr int kSigMaxN = 4096;
constexpr int kSigWork = 18;  // work vectors of n doubles per signal

struct SignalArgs {
    int n;          // samples
    int wk;         // half-width of the H^T H band (2m)
    int wt;         // half-width of the H^T band (m)
    int precond;    // TVD_PREC_*
    int wrap;       // periodic BCs: band columns wrap around (circulant)
    int max_outer, max_inner;
    double alpha, beta, inner_tol, fp_tol;
    const double* K;     // n x (2 wk + 1)
    const double* HT;    // n x (2 wt + 1)
    const double* Phi;   // n x n, Phi[i*n + k] = phi_k(i)
    const double* PhiT;  // n x n, PhiT[k*n + i] = phi_k(i)
    const double* lamh2; // n
    const double* v;     // observed signal
    double* u;           // restored signal
    double* work;        // kSigWork n
    // reblurring system (eq. (fpp), anti-reflective only): PBiCGstab with the
    // preconditioners of Section 3 in the algebra of T_n
    int reblur;          // 0: normal equations (PCG), 1: reblurring system (PBiCGstab)
    const double* HH;    // n x (2 wk + 1), band of H H
    const double* Hb;    // n x (2 wt + 1), band of H (b = H' v = H v)
    const double* TiT;   // n x n, TiT[i*n + k] = (T_n^{-1})[k][i]
    const double* TT;    // n x n, TT[k*n + i] = T_n[i][k]
    const double* wend;  // n - 2 end weights of AR(.)
    const int* replay;   // NULL, or max_outer iteration counts
    int* iters;          // max_outer
    double* relres;      // max_outer
    double* fpch;        // max_outer
    int* flags;          // [outer_steps, breakdown, all_converged]
};

__device__ __forceinline__ double sig_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();  // red is free: every thread has read the last sum
    if (lane == 0) red[w] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// y_i = sum_d band[i][d] x_{i+d}: the band of a matrix with the BC folded
// in; for periodic BCs column i + d wraps around (the band then holds the
// circulant's wrapped entries and 2w + 1 <= n).
__device__ __forceinline__ double sig_band_row(const double* row, const double* x, int i, int n, int w, int wrap) {
    double acc = 0.0;
    if (wrap) {
        for (int d = -w; d <= w; ++d) {
            int j = i + d;
            j += j < 0 ? n : 0;
            j -= j >= n ? n : 0;
            acc += row[d + w] * x[j];
        }
        return acc;
    }
    const int d0 = max(-w, -i), d1 = min(w, n - 1 - i);
    for (int d = d0; d <= d1; ++d) acc += row[d + w] * x[i + d];
    return acc;
}

// q = (H^T H + alpha L) p with the band of H^T H and the zero-Neumann
// stencil of the cell diffusivity kap (cell i couples samples i and i+1).
__device__ __forceinline__ void sig_apply_a(const SignalArgs& a, const double* kap, const double* p, double* q) {
    const int n = a.n, w = a.wk, bw = 2 * w + 1;
    for (int i = threadIdx.x; i < n; i += kSigThreads) {
        const double acc = sig_band_row(a.K + size_t(i) * bw, p, i, n, w, a.wrap);
        double lp = 0.0;
        if (i > 0) lp += kap[i - 1] * (p[i] - p[i - 1]);
        if (i < n - 1) lp -= kap[i] * (p[i + 1] - p[i]);
        q[i] = acc + a.alpha * lp;
    }
}

// z = P^{-1} r for the preconditioner of the current step: I, D
// (z = r / D), or s o Phi [(Phi^T (s o r)) / mu] for X, D_X, X_D.  t and y are
// n-double LDS vectors.
__device__ __forceinline__ void sig_precond(const SignalArgs& a, const double* r, const double* s, const double* dd,
                                            const double* minv, double* z, double* t, double* y) {
    const int n = a.n;
    if (a.precond == TVD_PREC_NONE) {
        for (int i = threadIdx.x; i < n; i += kSigThreads) z[i] = r[i];
        return;
    }
    if (a.precond == TVD_PREC_DIAG) {
        for (int i = threadIdx.x; i < n; i += kSigThreads) z[i] = r[i] / dd[i];
        return;
    }
    for (int i = threadIdx.x; i < n; i += kSigThreads) t[i] = s[i] * r[i];
    __syncthreads();
    // forward: y_k = sum_i phi_k(i) t_i (lanes over k read Phi rows coalesced)
    for (int k = threadIdx.x; k < n; k += kSigThreads) {
        double acc = 0.0;
        for (int i = 0; i < n; ++i) acc += a.Phi[size_t(i) * n + k] * t[i];
        y[k] = acc * minv[k];
    }
    __syncthreads();
    // inverse: z_i = s_i sum_k phi_k(i) y_k
    for (int i = threadIdx.x; i < n; i += kSigThreads) {
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += a.PhiT[size_t(k) * n + i] * y[k];
        z[i] = s[i] * acc;
    }
}

// q = (H H + alpha L) p, the matrix of eq. (fpp) (H' = H for a symmetric PSF).
__device__ __forceinline__ void sig_apply_reblur(const SignalArgs& a, const double* kap, const double* p, double* q) {
    const int n = a.n, w = a.wk, bw = 2 * w + 1;
    for (int i = threadIdx.x; i < n; i += kSigThreads) {
        const double acc = sig_band_row(a.HH + size_t(i) * bw, p, i, n, w, 0);
        double lp = 0.0;
        if (i > 0) lp += kap[i - 1] * (p[i] - p[i - 1]);
        if (i < n - 1) lp -= kap[i] * (p[i + 1] - p[i]);
        q[i] = acc + a.alpha * lp;
    }
}

// z = M^{-1} r for the reblurring system: I, D, or s o T [(T^{-1}(s o r)) / mu]
// for P, D_P, P_D (Section 3).
__device__ __forceinline__ void sig_precond_reblur(const SignalArgs& a, const double* r, const double* s,
                                                   const double* dd, const double* minv, double* z, double* t,
                                                   double* y) {
    const int n = a.n;
    if (a.precond == TVD_PREC_NONE) {
        for (int i = threadIdx.x; i < n; i += kSigThreads) z[i] = r[i];
        return;
    }
    if (a.precond == TVD_PREC_DIAG) {
        for (int i = threadIdx.x; i < n; i += kSigThreads) z[i] = r[i] / dd[i];
        return;
    }
    for (int i = threadIdx.x; i < n; i += kSigThreads) t[i] = s[i] * r[i];
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += kSigThreads) {
        double acc = 0.0;
        for (int i = 0; i < n; ++i) acc += a.TiT[size_t(i) * n + k] * t[i];
        y[k] = acc * minv[k];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kSigThreads) {
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += a.TT[size_t(k) * n + i] * y[k];
        z[i] = s[i] * acc;
    }
}

__global__ void __launch_bounds__(kSigThreads) k_signal(const SignalArgs* __restrict__ all) {
    const SignalArgs a = all[blockIdx.x];
    extern __shared__ double lds[];
    __shared__ double red[4];
    const int n = a.n, tid = threadIdx.x;
    double* t = lds;      // n
    double* y = lds + n;  // n
    double* W = a.work;
    double *x = W, *r = W + n, *p = W + 2 * n, *q = W + 3 * n, *z = W + 4 * n, *u = W + 5 * n, *b = W + 6 * n;
    double *kap = W + 7 * n, *s = W + 8 * n, *dd = W + 9 * n, *minv = W + 10 * n;
    double *rhat = W + 11 * n, *vv = W + 12 * n, *sv = W + 13 * n, *tv = W + 14 * n, *phat = W + 15 * n,
           *shat = W + 16 * n, *lam = W + 17 * n;
    const bool transform = a.precond >= TVD_PREC_X;
    const bool scaled = a.precond == TVD_PREC_D_X || a.precond == TVD_PREC_X_D;

    // b = H^T v, u^0 = v
    {
        const int w = a.wt, bw = 2 * w + 1;
        const double* B = a.reblur ? a.Hb : a.HT;
        for (int i = tid; i < n; i += kSigThreads) {
            b[i] = sig_band_row(B + size_t(i) * bw, a.v, i, n, w, a.wrap);
            u[i] = a.v[i];
        }
    }
    __syncthreads();
    int steps = 0, breakdown = 0, converged_all = 1;
    for (int k = 0; k < a.max_outer && !breakdown; ++k) {
        // diffusivity, D, scaling (cell i: forward difference u_{i+1} - u_i,
        // zero on the last cell)
        for (int i = tid; i < n; i += kSigThreads) {
            const double g = i < n - 1 ? u[i + 1] - u[i] : 0.0;
            kap[i] = 1.0 / sqrt(g * g + a.beta * a.beta);
        }
        __syncthreads();
        for (int i = tid; i < n; i += kSigThreads) {
            const double dl = (i < n - 1 ? kap[i] : 0.0) + (i > 0 ? kap[i - 1] : 0.0);
            dd[i] = 1.0 + a.alpha * dl;
            s[i] = scaled ? 1.0 / sqrt(dd[i]) : 1.0;
        }
        __syncthreads();
        // eigenvalues of the level-2 projection: mu_k = lam_H^2 + alpha lam_L
        // (X, D_X) or lam_H^2 lam_D^2 + alpha lam_L~ (X_D), Section 3
        if (transform && a.reblur) {
            // P, D_P, P_D: the interior eigenvalues are those of the S^
            // projection (interior frequencies 1..n-2), the two y = 0 ends
            // follow from them through the end weights of AR(.)
            const bool pd = a.precond == TVD_PREC_X_D;
            for (int kk = tid; kk < n; kk += kSigThreads) {
                double lam_l = 0.0, lam_d = 0.0;
                if (kk > 0 && kk < n - 1) {
                    double prev = a.Phi[kk] * (pd ? s[0] : 1.0);
                    if (pd) lam_d = s[0] * a.Phi[kk] * a.Phi[kk];
                    for (int i = 0; i < n - 1; ++i) {
                        const double ph = a.Phi[size_t(i + 1) * n + kk];
                        const double cur = ph * (pd ? s[i + 1] : 1.0);
                        const double d = cur - prev;
                        lam_l += kap[i] * d * d;
                        if (pd) lam_d += s[i + 1] * ph * ph;
                        prev = cur;
                    }
                }
                lam[kk] = lam_l;
                minv[kk] = lam_d;  // lam_D until the ends are known
            }
            __syncthreads();
            double el = 0.0, ed = 0.0;
            for (int j = tid; j < n - 2; j += kSigThreads) {
                el += a.wend[j] * lam[j + 1];
                ed += a.wend[j] * minv[j + 1];
            }
            el = sig_sum(el, red);
            ed = sig_sum(ed, red);
            for (int kk = tid; kk < n; kk += kSigThreads) {
                const bool end = kk == 0 || kk == n - 1;
                const double ll = end ? el : lam[kk];
                const double ld = end ? ed : minv[kk];
                const double mu = pd ? a.lamh2[kk] * ld * ld + a.alpha * ll : a.lamh2[kk] + a.alpha * ll;
                minv[kk] = 1.0 / mu;
            }
            __syncthreads();
        } else if (transform) {
            const bool xd = a.precond == TVD_PREC_X_D;
            for (int kk = tid; kk < n; kk += kSigThreads) {
                double lam_l = 0.0, lam_d = 0.0;
                double prev = a.Phi[kk] * (xd ? s[0] : 1.0);
                if (xd) lam_d = s[0] * a.Phi[kk] * a.Phi[kk];
                for (int i = 0; i < n - 1; ++i) {
                    const double ph = a.Phi[size_t(i + 1) * n + kk];
                    const double cur = ph * (xd ? s[i + 1] : 1.0);
                    const double d = cur - prev;
                    lam_l += kap[i] * d * d;
                    if (xd) lam_d += s[i + 1] * ph * ph;
                    prev = cur;
                }
                const double mu = xd ? a.lamh2[kk] * lam_d * lam_d + a.alpha * lam_l : a.lamh2[kk] + a.alpha * lam_l;
                minv[kk] = 1.0 / mu;
            }
            __syncthreads();
        }
        int it = 0;
        double relres = 1.0;
        bool conv = false;
        const int limit = a.replay ? a.replay[k] : a.max_inner;
        const double tol = a.replay ? 0.0 : a.inner_tol;
        for (int i = tid; i < n; i += kSigThreads) x[i] = u[i];
        __syncthreads();
        if (a.reblur) {
            // PBiCGstab (van der Vorst) from x_0 = u^k, shadow residual r_0,
            // the test ||r|| < tol ||r_0|| once per iteration
            sig_apply_reblur(a, kap, x, q);
            __syncthreads();
            double rr = 0.0;
            for (int i = tid; i < n; i += kSigThreads) {
                r[i] = b[i] - q[i];
                rhat[i] = r[i];
                p[i] = 0.0;
                vv[i] = 0.0;
                rr += r[i] * r[i];
            }
            const double r0 = sqrt(sig_sum(rr, red));
            relres = r0 == 0.0 ? 0.0 : 1.0;
            conv = r0 == 0.0;
            double rho_old = 1.0, al = 1.0, om = 1.0;
            while (r0 != 0.0 && it < limit) {
                double rp = 0.0;
                for (int i = tid; i < n; i += kSigThreads) rp += rhat[i] * r[i];
                const double rho = sig_sum(rp, red);
                if (rho == 0.0) {
                    breakdown = 1;
                    break;
                }
                const double bt = (rho / rho_old) * (al / om);
                for (int i = tid; i < n; i += kSigThreads) p[i] = r[i] + bt * (p[i] - om * vv[i]);
                __syncthreads();
                sig_precond_reblur(a, p, s, dd, minv, phat, t, y);
                __syncthreads();
                sig_apply_reblur(a, kap, phat, vv);
                __syncthreads();
                double sg = 0.0;
                for (int i = tid; i < n; i += kSigThreads) sg += rhat[i] * vv[i];
                const double sigma = sig_sum(sg, red);
                if (sigma == 0.0) {
                    breakdown = 1;
                    break;
                }
                al = rho / sigma;
                for (int i = tid; i < n; i += kSigThreads) sv[i] = r[i] - al * vv[i];
                __syncthreads();
                sig_precond_reblur(a, sv, s, dd, minv, shat, t, y);
                __syncthreads();
                sig_apply_reblur(a, kap, shat, tv);
                __syncthreads();
                double tt = 0.0, ts = 0.0;
                for (int i = tid; i < n; i += kSigThreads) {
                    tt += tv[i] * tv[i];
                    ts += tv[i] * sv[i];
                }
                tt = sig_sum(tt, red);
                ts = sig_sum(ts, red);
                om = tt > 0.0 ? ts / tt : 0.0;
                double rn2 = 0.0;
                for (int i = tid; i < n; i += kSigThreads) {
                    x[i] += al * phat[i] + om * shat[i];
                    r[i] = sv[i] - om * tv[i];
                    rn2 += r[i] * r[i];
                }
                ++it;
                const double rn = sqrt(sig_sum(rn2, red));
                relres = rn / r0;
                if (!a.replay && rn < tol * r0) {
                    conv = true;
                    break;
                }
                if (om == 0.0) {
                    breakdown = rn > 0.0 ? 1 : 0;
                    break;
                }
                rho_old = rho;
            }
        } else {
        // PCG (Golub-Van Loan 10.3.1) from x_0 = u^k
        sig_apply_a(a, kap, x, q);
        __syncthreads();
        double rr = 0.0;
        for (int i = tid; i < n; i += kSigThreads) {
            r[i] = b[i] - q[i];
            rr += r[i] * r[i];
        }
        const double r0 = sqrt(sig_sum(rr, red));
        relres = r0 == 0.0 ? 0.0 : 1.0;
        conv = r0 == 0.0;
        if (r0 != 0.0 && limit > 0) {
            sig_precond(a, r, s, dd, minv, z, t, y);
            __syncthreads();
            double rz = 0.0;
            for (int i = tid; i < n; i += kSigThreads) {
                p[i] = z[i];
                rz += r[i] * z[i];
            }
            double rho = sig_sum(rz, red);
            while (it < limit) {
                sig_apply_a(a, kap, p, q);
                __syncthreads();
                double pq = 0.0;
                for (int i = tid; i < n; i += kSigThreads) pq += p[i] * q[i];
                const double gamma = sig_sum(pq, red);
                ++it;
                if (!(gamma > 0.0)) {
                    --it;
                    breakdown = 1;
                    break;
                }
                const double al = rho / gamma;
                double rn2 = 0.0;
                for (int i = tid; i < n; i += kSigThreads) {
                    x[i] += al * p[i];
                    r[i] -= al * q[i];
                    rn2 += r[i] * r[i];
                }
                const double rn = sqrt(sig_sum(rn2, red));
                relres = rn / r0;
                if (!a.replay && rn < tol * r0) {
                    conv = true;
                    break;
                }
                if (it == limit) break;
                sig_precond(a, r, s, dd, minv, z, t, y);
                __syncthreads();
                double rz2 = 0.0;
                for (int i = tid; i < n; i += kSigThreads) rz2 += r[i] * z[i];
                const double rho2 = sig_sum(rz2, red);
                const double bt = rho2 / rho;
                for (int i = tid; i < n; i += kSigThreads) p[i] = z[i] + bt * p[i];
                rho = rho2;
                __syncthreads();
            }
        }
        }
        __syncthreads();
        // fixed-point change ||u^{k+1} - u^k|| / ||u^{k+1}||, u^{k+1} = x
        double dn = 0.0, xn = 0.0;
        for (int i = tid; i < n; i += kSigThreads) {
            const double d = x[i] - u[i];
            dn += d * d;
            xn += x[i] * x[i];
        }
        dn = sig_sum(dn, red);
        xn = sig_sum(xn, red);
        const double change = sqrt(dn) / fmax(sqrt(xn), 1e-300);
        for (int i = tid; i < n; i += kSigThreads) u[i] = x[i];
        if (!conv && !a.replay && it >= limit) converged_all = 0;
        if (breakdown) converged_all = 0;
        if (tid == 0) {
            a.iters[k] = it;
            a.relres[k] = relres;
            a.fpch[k] = change;
        }
        steps = k + 1;
        __syncthreads();
        if (a.fp_tol > 0.0 && change < a.fp_tol) break;
    }
    for (int i = tid; i < n; i += kSigThreads) a.u[i] = u[i];
    if (tid == 0) {
        a.flags[0] = steps;
        a.flags[1] = breakdown;
        a.flags[2] = converged_all;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side: per-signal tables, one device arena, one launch per solve.
struct SigError {
    hipError_t e;
    const char* what;
};
inline void sig_check(hipError_t e, const char* what) {
    if (e != hipSuccess) throw SigError{e, what};
}
#define TVD_SIG_HIP(expr) ::tvd::sig_check((expr), #expr)

class SignalBatch {
   public:
    SignalBatch(int count, hipStream_t s) : count_(count), s_(s) {}
    ~SignalBatch() { release(); }

    void build(const tvd_signal_desc* descs) {
        std::vector<double> tables;
        auto put = [&](const std::vector<double>& v) {
            size_t off = tables.size();
            tables.insert(tables.end(), v.begin(), v.end());
            while (tables.size() % 32) tables.push_back(0.0);  // 256-byte alignment
            return off;
        };
        sig_.resize(count_);
        size_t work = 0, total_n = 0;
        for (int i = 0; i < count_; ++i) {
            const tvd_signal_desc& d = descs[i];
            Sig& g = sig_[i];
            g.n = d.n;
            g.m = d.plen / 2;
            g.bc = d.bc;
            g.off_n = total_n;
            total_n += size_t(d.n);
            std::vector<double> h(d.psf_host, d.psf_host + d.plen);
            const std::vector<double> H = blur_matrix_1d(h, d.n, d.bc);
            g.wrap = d.bc == TVD_BC_PERIODIC ? 1 : 0;
            auto band = [&](const std::vector<double>& A, int w) {
                return g.wrap ? band_wrapped(A, d.n, w) : band_of(A, d.n, w);
            };
            g.K = put(band(matmul_tn(H, H, d.n), 2 * g.m));
            g.HT = put(band(transpose(H, d.n), g.m));
            const std::vector<double> Phi = basis_matrix(d.n, d.bc);
            g.Phi = put(Phi);
            g.PhiT = put(transpose(Phi, d.n));
            // the 1D symbol: row theta = 0 of the 2D symbol of the 1 x plen
            // PSF on a 3-row grid (a PSF of one row has the same value at
            // every row frequency)
            const std::vector<double> lam = symbol_eigenvalues(h.data(), 1, d.plen, 3, d.n, d.bc);
            std::vector<double> l2(d.n);
            for (int k = 0; k < d.n; ++k) l2[k] = lam[k] * lam[k];
            g.lamh2 = put(l2);
            g.reblur = d.reblur != 0;
            if (g.reblur) {  // the reblurring system's tables (anti-reflective only)
                g.HH = put(band_of(matmul_tn(transpose(H, d.n), H, d.n), d.n, 2 * g.m));
                g.Hb = put(band_of(H, d.n, g.m));
                std::vector<double> T, Ti;
                ar_transform_matrices(d.n, T, Ti);
                g.TiT = put(transpose(Ti, d.n));
                g.TT = put(transpose(T, d.n));
                g.wend = put(ar_end_weights(d.n));
            }
            g.work = work;
            work += size_t(kSigWork) * d.n + 32;
        }
        total_n_ = total_n;
        tables_ = static_cast<double*>(dalloc(tables.size() * sizeof(double)));
        TVD_SIG_HIP(hipMemcpyAsync(tables_, tables.data(), tables.size() * sizeof(double), hipMemcpyHostToDevice, s_));
        work_ = static_cast<double*>(dalloc(work * sizeof(double)));
        args_ = static_cast<SignalArgs*>(dalloc(count_ * sizeof(SignalArgs)));
        const int K = TVD_MAX_OUTER;
        iters_ = static_cast<int*>(dalloc(size_t(count_) * K * sizeof(int)));
        relres_ = static_cast<double*>(dalloc(size_t(count_) * K * sizeof(double)));
        fpch_ = static_cast<double*>(dalloc(size_t(count_) * K * sizeof(double)));
        flags_ = static_cast<int*>(dalloc(size_t(count_) * 4 * sizeof(int)));
        replay_ = static_cast<int*>(dalloc(size_t(count_) * K * sizeof(int)));
        TVD_SIG_HIP(hipStreamSynchronize(s_));
        max_n_ = 0;
        for (const Sig& g : sig_) max_n_ = std::max(max_n_, g.n);
    }

    void solve(const double* v, double* u, const tvd_signal_params& p, tvd_stats* stats) {
        const int K = TVD_MAX_OUTER;
        std::vector<SignalArgs> args(count_);
        if (p.replay_host) {
            std::vector<int> rp(size_t(count_) * K, 0);
            for (int i = 0; i < count_; ++i)
                for (int k = 0; k < p.max_outer; ++k) rp[size_t(i) * K + k] = p.replay_host[size_t(i) * p.max_outer + k];
            TVD_SIG_HIP(hipMemcpyAsync(replay_, rp.data(), rp.size() * sizeof(int), hipMemcpyHostToDevice, s_));
        }
        for (int i = 0; i < count_; ++i) {
            const Sig& g = sig_[i];
            SignalArgs& a = args[i];
            a.n = g.n;
            a.wk = 2 * g.m;
            a.wt = g.m;
            a.precond = p.precond_host ? p.precond_host[i] : p.precond;
            a.wrap = g.wrap;
            a.reblur = (p.system_host ? p.system_host[i] : p.system) != 0;
            if (a.reblur) {
                a.HH = tables_ + g.HH;
                a.Hb = tables_ + g.Hb;
                a.TiT = tables_ + g.TiT;
                a.TT = tables_ + g.TT;
                a.wend = tables_ + g.wend;
            }
            a.max_outer = p.max_outer;
            a.max_inner = p.max_inner;
            a.alpha = p.alpha_host[i];
            a.beta = p.beta_host ? p.beta_host[i] : p.beta;
            a.inner_tol = p.inner_tol;
            a.fp_tol = p.fp_tol;
            a.K = tables_ + g.K;
            a.HT = tables_ + g.HT;
            a.Phi = tables_ + g.Phi;
            a.PhiT = tables_ + g.PhiT;
            a.lamh2 = tables_ + g.lamh2;
            a.v = v + g.off_n;
            a.u = u + g.off_n;
            a.work = work_ + g.work;
            a.replay = p.replay_host ? replay_ + size_t(i) * K : nullptr;
            a.iters = iters_ + size_t(i) * K;
            a.relres = relres_ + size_t(i) * K;
            a.fpch = fpch_ + size_t(i) * K;
            a.flags = flags_ + size_t(i) * 4;
        }
        TVD_SIG_HIP(hipMemcpyAsync(args_, args.data(), args.size() * sizeof(SignalArgs), hipMemcpyHostToDevice, s_));
        hipEvent_t e0, e1;
        TVD_SIG_HIP(hipEventCreate(&e0));
        TVD_SIG_HIP(hipEventCreate(&e1));
        TVD_SIG_HIP(hipEventRecord(e0, s_));
        hipLaunchKernelGGL(k_signal, dim3(count_), dim3(kSigThreads), size_t(2) * max_n_ * sizeof(double), s_,
                           static_cast<const SignalArgs*>(args_));
        TVD_SIG_HIP(hipGetLastError());
        TVD_SIG_HIP(hipEventRecord(e1, s_));
        std::vector<int> it(size_t(count_) * K), fl(size_t(count_) * 4);
        std::vector<double> rr(size_t(count_) * K), fc(size_t(count_) * K);
        TVD_SIG_HIP(hipMemcpyAsync(it.data(), iters_, it.size() * sizeof(int), hipMemcpyDeviceToHost, s_));
        TVD_SIG_HIP(hipMemcpyAsync(rr.data(), relres_, rr.size() * sizeof(double), hipMemcpyDeviceToHost, s_));
        TVD_SIG_HIP(hipMemcpyAsync(fc.data(), fpch_, fc.size() * sizeof(double), hipMemcpyDeviceToHost, s_));
        TVD_SIG_HIP(hipMemcpyAsync(fl.data(), flags_, fl.size() * sizeof(int), hipMemcpyDeviceToHost, s_));
        TVD_SIG_HIP(hipStreamSynchronize(s_));
        float ms = 0.f;
        TVD_SIG_HIP(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        last_ms_ = ms;
        any_breakdown_ = false;
        for (int i = 0; i < count_; ++i) {
            const int steps = fl[size_t(i) * 4];
            if (fl[size_t(i) * 4 + 1]) any_breakdown_ = true;
            if (!stats) continue;
            tvd_stats& st = stats[i];
            std::memset(&st, 0, sizeof(st));
            st.outer_steps = steps;
            st.breakdown = fl[size_t(i) * 4 + 1];
            st.all_converged = fl[size_t(i) * 4 + 2];
            for (int k = 0; k < steps; ++k) {
                st.inner_iters[k] = it[size_t(i) * K + k];
                st.relres[k] = rr[size_t(i) * K + k];
                st.fp_change[k] = fc[size_t(i) * K + k];
                st.total_inner_iters += st.inner_iters[k];
            }
            st.time_total_s = ms * 1e-3;
            st.time_inner_s = ms * 1e-3;
        }
    }

    size_t total_n() const { return total_n_; }
    bool has_reblur(int i) const { return sig_[i].reblur; }
    int count() const { return count_; }
    bool breakdown() const { return any_breakdown_; }
    double last_ms() const { return last_ms_; }
    std::string err;

   private:
    struct Sig {
        int n = 0, m = 0, bc = 0, wrap = 0;
        bool reblur = false;
        size_t off_n = 0, K = 0, HT = 0, Phi = 0, PhiT = 0, lamh2 = 0, work = 0;
        size_t HH = 0, Hb = 0, TiT = 0, TT = 0, wend = 0;
    };
    void* dalloc(size_t bytes) {
        void* p = nullptr;
        const hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 16));
        if (e != hipSuccess) throw std::bad_alloc();
        ptrs_.push_back(p);
        return p;
    }
    void release() {
        for (void* p : ptrs_) (void)hipFree(p);
        ptrs_.clear();
    }

    int count_;
    hipStream_t s_;
    std::vector<Sig> sig_;
    std::vector<void*> ptrs_;
    double* tables_ = nullptr;
    double* work_ = nullptr;
    SignalArgs* args_ = nullptr;
    int *iters_ = nullptr, *flags_ = nullptr, *replay_ = nullptr;
    double *relres_ = nullptr, *fpch_ = nullptr;
    size_t total_n_ = 0;
    int max_n_ = 0;
    bool any_breakdown_ = false;
    double last_ms_ = 0.0;

   public:
    template <typename F>
    static int guarded(SignalBatch* b, std::string* err, F&& f) {
        try {
            return f();
        } catch (const SigError& e) {
            *err = std::string(e.what) + ": " + hipGetErrorString(e.e);
            return TVD_EDEVICE;
        } catch (const std::bad_alloc&) {
            *err = "allocation failed";
            return TVD_ENOMEM;
        } catch (...) {
            *err = "unexpected internal error";
            return TVD_EDEVICE;
        }
    }
};

}  // namespace tvd

struct tvdeblur_signals {
    std::unique_ptr<tvd::SignalBatch> b;
    std::string err;
};

namespace {
std::string g_signals_create_error;
std::mutex g_signals_mu;

int sfail(tvdeblur_signals_t s, int code, const std::string& msg) {
    if (s) s->err = msg;
    else {
        std::lock_guard<std::mutex> lk(g_signals_mu);
        g_signals_create_error = msg;
    }
    return code;
}
}  // namespace

extern "C" {

int tvdeblur_signals_create(tvdeblur_signals_t* out, int count, const tvd_signal_desc* descs, void* hip_stream) {
    if (!out) return sfail(nullptr, TVD_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || count > 65536 || !descs) return sfail(nullptr, TVD_EINVAL, "count must be 1..65536 with descs");
    for (int i = 0; i < count; ++i) {
        const tvd_signal_desc& d = descs[i];
        const std::string at = "signal " + std::to_string(i) + ": ";
        if (d.n < 3 || d.n > tvd::kSigMaxN)
            return sfail(nullptr, TVD_ESIZE, at + "n must be 3.." + std::to_string(tvd::kSigMaxN));
        if (d.bc < TVD_BC_REFLECTIVE || d.bc > TVD_BC_PERIODIC)
            return sfail(nullptr, TVD_EINVAL, at + "bad boundary condition");
        if (!d.psf_host) return sfail(nullptr, TVD_EINVAL, at + "NULL PSF");
        std::string e;
        const int rc = tvd::validate_psf(d.psf_host, 1, d.plen, e);
        if (rc == -1) return sfail(nullptr, TVD_EINVAL, at + e);
        if (rc == -2) return sfail(nullptr, TVD_ENOTSYM, at + e);
        if (rc == -3) return sfail(nullptr, TVD_ENORM, at + e);
        const int m = d.plen / 2;
        if ((d.bc == TVD_BC_ANTIREFLECTIVE && m > d.n - 1) || m > d.n)
            return sfail(nullptr, TVD_ESIZE, at + "PSF half-width too large for the signal");
        if (d.bc == TVD_BC_PERIODIC && 4 * m + 1 > d.n)
            return sfail(nullptr, TVD_ESIZE, at + "periodic BCs need 4m + 1 <= n (the wrapped band of H^T H)");
        if (d.reblur && d.bc != TVD_BC_ANTIREFLECTIVE)
            return sfail(nullptr, TVD_EINVAL, at + "the reblurring system needs anti-reflective BCs");
    }
    tvdeblur_signals_t s = new (std::nothrow) tvdeblur_signals();
    if (!s) return sfail(nullptr, TVD_ENOMEM, "host allocation failed");
    std::string err;
    const int rc = tvd::SignalBatch::guarded(nullptr, &err, [&]() {
        s->b.reset(new tvd::SignalBatch(count, static_cast<hipStream_t>(hip_stream)));
        s->b->build(descs);
        return TVD_OK;
    });
    if (rc != TVD_OK) {
        delete s;
        return sfail(nullptr, rc, err);
    }
    *out = s;
    return TVD_OK;
}

int tvdeblur_signals_solve(tvdeblur_signals_t s, const double* v_dev, double* u_dev, const tvd_signal_params* p,
                           tvd_stats* stats_host) {
    if (!s) return sfail(nullptr, TVD_EINVAL, "NULL handle");
    if (!v_dev || !u_dev || !p || !p->alpha_host) return sfail(s, TVD_EINVAL, "NULL argument");
    if (v_dev == u_dev) return sfail(s, TVD_EINVAL, "v and u must not alias");
    if (p->max_outer < 1 || p->max_outer > TVD_MAX_OUTER) return sfail(s, TVD_EINVAL, "max_outer out of range");
    if (p->max_inner < 1 || !(p->inner_tol >= 0) || !(p->fp_tol >= 0))
        return sfail(s, TVD_EINVAL, "bad inner_tol / max_inner / fp_tol");
    const int count = s->b->count();
    for (int i = 0; i < count; ++i) {
        const double a = p->alpha_host[i], bt = p->beta_host ? p->beta_host[i] : p->beta;
        const int pc = p->precond_host ? p->precond_host[i] : p->precond;
        if (!std::isfinite(a) || a < 0 || !std::isfinite(bt) || !(bt > 0))
            return sfail(s, TVD_EINVAL, "signal " + std::to_string(i) + ": alpha >= 0 and beta > 0, finite");
        if (pc < TVD_PREC_NONE || pc > TVD_PREC_X_D)
            return sfail(s, TVD_EINVAL, "signal " + std::to_string(i) + ": bad preconditioner");
        const int sys = p->system_host ? p->system_host[i] : p->system;
        if (sys != 0 && sys != 1) return sfail(s, TVD_EINVAL, "signal " + std::to_string(i) + ": bad system");
        if (sys == 1 && !s->b->has_reblur(i))
            return sfail(s, TVD_EINVAL,
                         "signal " + std::to_string(i) + ": reblurring system not built (tvd_signal_desc.reblur)");
    }
    if (p->replay_host)
        for (size_t k = 0; k < size_t(count) * p->max_outer; ++k)
            if (p->replay_host[k] < 0) return sfail(s, TVD_EINVAL, "negative replay count");
    std::string err;
    const int rc = tvd::SignalBatch::guarded(s->b.get(), &err, [&]() {
        s->b->solve(v_dev, u_dev, *p, stats_host);
        return s->b->breakdown() ? TVD_EBREAKDOWN : TVD_OK;
    });
    if (rc == TVD_EBREAKDOWN)
        return sfail(s, rc, "breakdown in at least one signal (PCG: p^T A p <= 0; BiCGstab: rho, <rhat, v> or omega 0)");
    if (rc != TVD_OK) return sfail(s, rc, err);
    return TVD_OK;
}

int tvdeblur_signals_destroy(tvdeblur_signals_t s) {
    delete s;
    return TVD_OK;
}

const char* tvdeblur_signals_last_error(tvdeblur_signals_t s) {
    if (s) return s->err.c_str();
    std::lock_guard<std::mutex> lk(g_signals_mu);
    return g_signals_create_error.c_str();
}

}  // extern "C"

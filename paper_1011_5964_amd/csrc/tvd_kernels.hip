// HIP kernels of libtvdeblur for CDNA4 (gfx950).
//
// Per PCG iteration of the fixed-point system (H^T H + alpha L(u^k)) u = H^T v
// (eq. (fp)) four kernels run:
//   band     p = z + beta p (fused), q = H^T H p + alpha L(u^k) p, <p,q> partials
//   rowpass0 x += a p, r -= a q, ||r||^2 partials, s o r, 1D transform of rows
//   colpass  convergence test, 1D transform of columns, divide by mu, inverse
//   rowpass1 inverse 1D transform of rows, z = s o ., <r,z> partials
// Reductions are per-block FP64 partial sums that the next kernel adds up in a
// fixed order (deterministic, no atomics); the CG scalars never leave the GPU.
#include "tvd_internal.hpp"

#include <hip/hip_runtime.h>

#include <cmath>

namespace tvd {

namespace {

constexpr int kWave = 64;
constexpr int kBandTX = 64;    // band tile width (one wavefront across a row)
constexpr int kBandTYMax = 16; // band tile height is 8 or 16 (runtime)
constexpr int kBandThreads = 256;

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) {
    return {a.x, -a.y};
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum of v over the block; every thread gets the result.  red: >= 17 doubles.
__device__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x < kWave) {
        double s = (threadIdx.x < nw) ? red[threadIdx.x] : 0.0;
        s = wave_sum(s);
        if (threadIdx.x == 0) red[16] = s;
    }
    __syncthreads();
    return red[16];
}

// Deterministic sum of n per-block partials, computed redundantly per block.
__device__ double sum_partials(const double* p, int n, double* red) {
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) s += p[k];
    return block_sum(s, red);
}

// ------------------------------------------------------------------------
// Banded Kronecker operator with LDS halo tile.
// out(i,j) = sum_r sum_di By_r[i][di] sum_dj Bx_r[j][dj] X(i+di, j+dj)
// The boundary condition of the blur is folded into the band coefficients,
// so the kernel only sees zeros outside the image.
// ------------------------------------------------------------------------
template <typename TX, typename TS, typename T, typename TOut>
__global__ void __launch_bounds__(kBandThreads) k_band(BandArgsT<TX, TS, T, TOut> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[17];
    if (a.st && a.st->done) return;

    const int tid = threadIdx.x;
    const int tx = tid & (kBandTX - 1);
    const int ty = tid / kBandTX;            // 0..3
    const int TY = a.tile_y;
    const int i0 = blockIdx.y * TY;
    const int j0 = blockIdx.x * kBandTX;
    const int ny = a.ny, nx = a.nx;
    const bool stencil = a.kap != nullptr;
    const bool sten_tile = stencil && a.S == nullptr;
    const int hy = max(a.wy, sten_tile ? 1 : 0);
    const int hx = max(a.wx, sten_tile ? 1 : 0);
    const int PH = TY + 2 * hy, PW = kBandTX + 2 * hx;
    const int TH = TY + 2 * a.wy;
    const int by_w = 2 * a.wy + 1, bx_w = 2 * a.wx + 1;

    T* P = reinterpret_cast<T*>(smem_raw);
    T* tmp = P + PH * PW;
    T* bxl = tmp + TH * kBandTX;                       // [nterms][TX][bx_w]
    T* byl = bxl + a.nterms * kBandTX * bx_w;           // [nterms][TY][by_w]
    T* Sl = byl + a.nterms * TY * by_w;            // [(TY+2)][(TX+2)] if separate stencil input

    // p-update coefficient from the <r,z> partials of the last two iterations
    T beta = T(0);
    const bool upd = a.Z != nullptr;
    const bool use_old = upd && a.rz_old != nullptr;
    if (use_old) {
        const double rn = sum_partials(a.rz_new, a.n_rz, red);
        const double ro = sum_partials(a.rz_old, a.n_rz, red);
        beta = T(rn / ro);
    }

    // stage input tile (zeros outside the image)
    for (int k = tid; k < PH * PW; k += kBandThreads) {
        const int r = k / PW, c = k - r * PW;
        const int gi = i0 - hy + r, gj = j0 - hx + c;
        T v = T(0);
        if (gi >= 0 && gi < ny && gj >= 0 && gj < nx) {
            const size_t g = size_t(gi) * nx + gj;
            if (upd) {
                TX w = a.Z[g];
                if (use_old) w += TX(beta) * a.X[g];
                if (r >= hy && r < hy + TY && c >= hx && c < hx + kBandTX) a.Xnew[g] = w;
                v = T(w);
            } else {
                v = T(a.X[g]);
            }
        }
        P[k] = v;
    }
    for (int k = tid; k < a.nterms * kBandTX * bx_w; k += kBandThreads) {
        const int r = k / (kBandTX * bx_w);
        const int rem = k - r * kBandTX * bx_w;
        const int c = rem / bx_w, d = rem - c * bx_w;
        const int gj = j0 + c;
        bxl[k] = (gj < nx) ? a.Bx[(size_t(r) * nx + gj) * bx_w + d] : T(0);
    }
    for (int k = tid; k < a.nterms * TY * by_w; k += kBandThreads) {
        const int r = k / (TY * by_w);
        const int rem = k - r * TY * by_w;
        const int c = rem / by_w, d = rem - c * by_w;
        const int gi = i0 + c;
        byl[k] = (gi < ny) ? a.By[(size_t(r) * ny + gi) * by_w + d] : T(0);
    }
    const bool sten_sep = stencil && a.S != nullptr;
    if (sten_sep) {
        const int SW = kBandTX + 2;
        for (int k = tid; k < (TY + 2) * SW; k += kBandThreads) {
            const int r = k / SW, c = k - r * SW;
            const int gi = i0 - 1 + r, gj = j0 - 1 + c;
            Sl[k] = (gi >= 0 && gi < ny && gj >= 0 && gj < nx) ? T(a.S[size_t(gi) * nx + gj]) : T(0);
        }
    }
    __syncthreads();

    T acc[kBandTYMax / 4];
#pragma unroll
    for (int k = 0; k < kBandTYMax / 4; ++k) acc[k] = T(0);
    const int nacc = TY / 4;

    for (int term = 0; term < a.nterms; ++term) {
        // row pass: tmp[lr][tx] = sum_d bx[tx][d] P[lr + hy - wy][hx + tx + d - wx]
        const T* bxr = bxl + (term * kBandTX + tx) * bx_w;
        for (int lr = ty; lr < TH; lr += 4) {
            const T* prow = P + (lr + hy - a.wy) * PW + (hx - a.wx) + tx;
            T s = T(0);
            for (int d = 0; d < bx_w; ++d) s += bxr[d] * prow[d];
            tmp[lr * kBandTX + tx] = s;
        }
        __syncthreads();
        // column pass
#pragma unroll
        for (int k = 0; k < kBandTYMax / 4; ++k) {
            if (k >= nacc) break;
            const int ti = ty + 4 * k;
            const T* byr = byl + (term * TY + ti) * by_w;
            const T* tcol = tmp + ti * kBandTX + tx;
            T s = T(0);
            for (int d = 0; d < by_w; ++d) s += byr[d] * tcol[d * kBandTX];
            acc[k] += s;
        }
        __syncthreads();
    }

    double dot = 0.0;
#pragma unroll
    for (int k = 0; k < kBandTYMax / 4; ++k) {
        if (k >= nacc) break;
        const int ti = ty + 4 * k;
        const int gi = i0 + ti, gj = j0 + tx;
        if (gi >= ny || gj >= nx) continue;
        const size_t g = size_t(gi) * nx + gj;
        T res = acc[k];
        T cen = T(0);
        if (stencil) {
            T up, dn, lf, rt;
            if (sten_tile) {
                const T* pc = P + (hy + ti) * PW + hx + tx;
                cen = pc[0];
                up = pc[-PW];
                dn = pc[PW];
                lf = pc[-1];
                rt = pc[1];
            } else {
                const int SW = kBandTX + 2;
                const T* pc = Sl + (ti + 1) * SW + tx + 1;
                cen = pc[0];
                up = pc[-SW];
                dn = pc[SW];
                lf = pc[-1];
                rt = pc[1];
            }
            const T kc = a.kap[g];
            T lp = T(0);
            if (gi > 0) lp += a.kap[g - nx] * (cen - up);
            if (gi < ny - 1) lp += kc * (cen - dn);
            if (gj > 0) lp += a.kap[g - 1] * (cen - lf);
            if (gj < nx - 1) lp += kc * (cen - rt);
            res += T(a.alpha) * lp;
        } else if (a.dotmode == 1) {
            cen = P[(hy + ti) * PW + hx + tx];
        }
        if (a.Bvec) res = a.Bvec[g] - res;
        const TOut out = TOut(res);
        a.Y[g] = out;
        if (a.dotmode == 1) dot += double(cen) * double(out);
        else if (a.dotmode == 2) dot += double(out) * double(out);
    }
    if (a.dotmode) {
        const double s = block_sum(dot, red);
        if (tid == 0) a.dot_part[blockIdx.y * gridDim.x + blockIdx.x] = s;
    }
}

// ------------------------------------------------------------------------
// Line transforms in LDS: two real lines packed as one complex sequence.
// ------------------------------------------------------------------------

// Stockham radix-2 FFT (forward, exp(-2 pi i/M)) of the unit's sequence,
// ping-ponging between x and y; returns the buffer holding the result.
template <typename T>
__device__ cx<T>* fft_pow2(cx<T>* x, cx<T>* y, int M, int log2M, const cx<T>* __restrict__ tw,
                           int lt, int tpu) {
    const int half = M >> 1;
    int s = 1;
    for (int st = 0; st < log2M; ++st) {
        for (int b = lt; b < half; b += tpu) {
            const int p = b >> st, q = b & (s - 1);
            const cx<T> u = x[b], v = x[b + half];
            const cx<T> w = tw[p * s];
            const cx<T> d = {u.x - v.x, u.y - v.y};
            y[q + 2 * s * p] = {u.x + v.x, u.y + v.y};
            y[q + s * (2 * p + 1)] = cmul(d, w);
        }
        __syncthreads();
        cx<T>* t = x;
        x = y;
        y = t;
        s <<= 1;
    }
    return x;
}

// Full DFT of length L of buffer b0 (already assembled; Bluestein inputs are
// chirp-multiplied and zero padded to M).  Returns the result buffer; the
// caller reads X_k through dft_get().
template <typename T>
__device__ cx<T>* dft_run(cx<T>* b0, cx<T>* b1, const AxisPlan<T>& P, int lt, int tpu) {
    cx<T>* r = fft_pow2(b0, b1, P.M, P.log2M, P.tw, lt, tpu);
    if (!P.bluestein) return r;
    cx<T>* o = (r == b0) ? b1 : b0;
    for (int k = lt; k < P.M; k += tpu) r[k] = cconj(cmul(r[k], P.bf[k]));
    __syncthreads();
    return fft_pow2(r, o, P.M, P.log2M, P.tw, lt, tpu);
}

template <typename T>
__device__ __forceinline__ cx<T> dft_get(const cx<T>* r, int k, const AxisPlan<T>& P) {
    if (!P.bluestein) return r[k];
    return cmul(P.chirp[k], cconj(r[k]));
}

template <typename T>
__device__ __forceinline__ void dft_put(cx<T>* b, int t, cx<T> v, const AxisPlan<T>& P) {
    b[t] = P.bluestein ? cmul(v, P.chirp[t]) : v;
}

template <typename T>
__device__ __forceinline__ void dft_pad(cx<T>* b, const AxisPlan<T>& P, int lt, int tpu) {
    if (P.bluestein)
        for (int t = P.L + lt; t < P.M; t += tpu) b[t] = {T(0), T(0)};
}

// Assemble the forward transform input for position t of the two lines
// (value v = a + i b).  DST-I: odd extension of the interior; DCT-II: even
// extension.  Positions 0 and n-1 of a DST line are pass-through and get 0.
template <typename T>
__device__ __forceinline__ void put_forward(cx<T>* b, int t, cx<T> v, const AxisPlan<T>& P) {
    const int n = P.n;
    if (P.kind == 1) {
        if (t == 0 || t == n - 1) {
            dft_put(b, t, cx<T>{T(0), T(0)}, P);
        } else {
            dft_put(b, t, v, P);
            dft_put(b, P.L - t, cx<T>{-v.x, -v.y}, P);
        }
    } else {
        dft_put(b, t, v, P);
        dft_put(b, 2 * n - 1 - t, v, P);
    }
}

// Assemble the inverse transform input from coefficient k (value v).
// DST-I is its own inverse.  DCT-III: Hermitian extension of the weighted
// coefficients, conjugated so that the forward DFT computes the inverse.
template <typename T>
__device__ __forceinline__ void put_inverse(cx<T>* b, int k, cx<T> v, const AxisPlan<T>& P) {
    if (P.kind == 1) {
        put_forward(b, k, v, P);
        return;
    }
    const int n = P.n;
    const cx<T> w = P.pre[k];
    if (k == 0) {
        const cx<T> y0 = {T(2) * w.x * v.x, T(2) * w.x * v.y};
        dft_put(b, 0, cconj(y0), P);
        dft_put(b, n, cx<T>{T(0), T(0)}, P);
    } else {
        dft_put(b, k, cconj(cmul(w, v)), P);
        dft_put(b, 2 * n - k, cconj(cmul(cconj(w), v)), P);
    }
}

// Read forward output at position/frequency k as the two real results.
template <typename T>
__device__ __forceinline__ cx<T> get_forward(const cx<T>* r, int k, const AxisPlan<T>& P) {
    const cx<T> F = dft_get(r, k, P);
    if (P.kind == 1) return {-F.y * P.dst_scale, F.x * P.dst_scale};
    return cmul(F, P.post[k]);
}

template <typename T>
__device__ __forceinline__ cx<T> get_inverse(const cx<T>* r, int t, const AxisPlan<T>& P) {
    if (P.kind == 1) return get_forward(r, t, P);
    const cx<T> G = cconj(dft_get(r, t, P));
    return {G.x * T(0.5), G.y * T(0.5)};
}

template <typename T>
__device__ __forceinline__ bool passthrough(int t, const AxisPlan<T>& P) {
    return P.kind == 1 && (t == 0 || t == P.n - 1);
}

// Row pass.  mode 0: (optional x,r update) then T1 = Qx (s o r) row-wise.
//            mode 1: z = s o (Qx^T T2) row-wise, <r, z> partials.
template <typename T>
__global__ void k_rowpass(RowPassArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[17];
    if (a.st->done) return;
    const AxisPlan<T>& P = a.plan;
    const int tid = threadIdx.x;
    const int ul = tid / a.g.tpu, lt = tid - ul * a.g.tpu;
    const int unit = blockIdx.x * a.g.upb + ul;
    const int nx = a.nx, ny = a.ny;
    cx<T>* b0 = reinterpret_cast<cx<T>*>(smem_raw) + size_t(ul) * 2 * P.M;
    cx<T>* b1 = b0 + P.M;
    const int ia = 2 * unit, ib = 2 * unit + 1;
    const bool va = ia < ny, vb = ib < ny;

    double part = 0.0;
    if (a.mode == 0) {
        T step = T(0);
        if (a.do_update) {
            const double g = sum_partials(a.pq_part, a.n_pq, red);
            const double rz = sum_partials(a.rz_part, a.n_rz, red);
            if (!(g > 0.0)) {  // curvature <= 0 (or NaN): stop, keep x_{i-1}
                if (blockIdx.x == 0 && tid == 0) {
                    a.st->done = 2;
                    a.st->iters = a.iter - 1;
                }
                return;
            }
            step = T(rz / g);
        }
        for (int t = lt; t < nx; t += a.g.tpu) {
            T ra = T(0), rb = T(0);
            if (va) {
                const size_t g = size_t(ia) * nx + t;
                ra = a.r[g];
                if (a.do_update) {
                    a.x[g] += step * a.p[g];
                    ra -= step * a.q[g];
                    a.r[g] = ra;
                    part += double(ra) * double(ra);
                }
                if (a.s) ra *= a.s[g];
            }
            if (vb) {
                const size_t g = size_t(ib) * nx + t;
                rb = a.r[g];
                if (a.do_update) {
                    a.x[g] += step * a.p[g];
                    rb -= step * a.q[g];
                    a.r[g] = rb;
                    part += double(rb) * double(rb);
                }
                if (a.s) rb *= a.s[g];
            }
            if (passthrough(t, P)) {
                if (va) a.dst[size_t(ia) * nx + t] = ra;
                if (vb) a.dst[size_t(ib) * nx + t] = rb;
            }
            put_forward(b0, t, cx<T>{ra, rb}, P);
        }
        dft_pad(b0, P, lt, a.g.tpu);
        __syncthreads();
        cx<T>* res = dft_run(b0, b1, P, lt, a.g.tpu);
        for (int k = lt; k < nx; k += a.g.tpu) {
            if (passthrough(k, P)) continue;
            const cx<T> o = get_forward(res, k, P);
            if (va) a.dst[size_t(ia) * nx + k] = o.x;
            if (vb) a.dst[size_t(ib) * nx + k] = o.y;
        }
        if (a.do_update) {
            const double s = block_sum(part, red);
            if (tid == 0) a.part_out[blockIdx.x] = s;
        }
    } else {
        for (int k = lt; k < nx; k += a.g.tpu) {
            const T ya = va ? a.src[size_t(ia) * nx + k] : T(0);
            const T yb = vb ? a.src[size_t(ib) * nx + k] : T(0);
            if (passthrough(k, P)) {
                if (va) {
                    const size_t g = size_t(ia) * nx + k;
                    const T z = a.s ? a.s[g] * ya : ya;
                    a.dst[g] = z;
                    part += double(a.r[g]) * double(z);
                }
                if (vb) {
                    const size_t g = size_t(ib) * nx + k;
                    const T z = a.s ? a.s[g] * yb : yb;
                    a.dst[g] = z;
                    part += double(a.r[g]) * double(z);
                }
            }
            put_inverse(b0, k, cx<T>{ya, yb}, P);
        }
        dft_pad(b0, P, lt, a.g.tpu);
        __syncthreads();
        cx<T>* res = dft_run(b0, b1, P, lt, a.g.tpu);
        for (int t = lt; t < nx; t += a.g.tpu) {
            if (passthrough(t, P)) continue;
            const cx<T> o = get_inverse(res, t, P);
            if (va) {
                const size_t g = size_t(ia) * nx + t;
                const T z = a.s ? a.s[g] * o.x : o.x;
                a.dst[g] = z;
                part += double(a.r[g]) * double(z);
            }
            if (vb) {
                const size_t g = size_t(ib) * nx + t;
                const T z = a.s ? a.s[g] * o.y : o.y;
                a.dst[g] = z;
                part += double(a.r[g]) * double(z);
            }
        }
        const double s = block_sum(part, red);
        if (tid == 0) a.part_out[blockIdx.x] = s;
    }
}

// Column pass: convergence test, forward column transform, divide by mu,
// inverse column transform.
template <typename T>
__global__ void k_colpass(ColPassArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[17];
    if (a.st->done) return;
    if (a.check) {
        const double rn = sqrt(sum_partials(a.rr_part, a.n_rr, red));
        if (a.iter == 0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                a.st->r0norm = rn;
                a.st->relres = rn > 0.0 ? 1.0 : 0.0;
                if (rn == 0.0) {
                    a.st->done = 1;
                    a.st->iters = 0;
                }
            }
            if (rn == 0.0) return;
        } else {
            const double r0 = a.st->r0norm;
            if (blockIdx.x == 0 && threadIdx.x == 0) a.st->relres = rn / r0;
            if (rn < a.st->tol * r0) {
                if (blockIdx.x == 0 && threadIdx.x == 0) {
                    a.st->done = 1;
                    a.st->iters = a.iter;
                }
                return;
            }
        }
    }
    const AxisPlan<T>& P = a.plan;
    const int tid = threadIdx.x;
    const int ul = tid / a.g.tpu, lt = tid - ul * a.g.tpu;
    const int unit = blockIdx.x * a.g.upb + ul;
    const int nx = a.nx, ny = a.ny;
    cx<T>* b0 = reinterpret_cast<cx<T>*>(smem_raw) + size_t(ul) * 2 * P.M;
    cx<T>* b1 = b0 + P.M;
    const int ja = 2 * unit, jb = 2 * unit + 1;
    const bool va = ja < nx, vb = jb < nx;

    for (int t = lt; t < ny; t += a.g.tpu) {
        const T xa = va ? a.src[size_t(t) * nx + ja] : T(0);
        const T xb = vb ? a.src[size_t(t) * nx + jb] : T(0);
        if (passthrough(t, P)) {
            if (va) a.dst[size_t(t) * nx + ja] = xa * a.muinv[size_t(t) * nx + ja];
            if (vb) a.dst[size_t(t) * nx + jb] = xb * a.muinv[size_t(t) * nx + jb];
        }
        put_forward(b0, t, cx<T>{xa, xb}, P);
    }
    dft_pad(b0, P, lt, a.g.tpu);
    __syncthreads();
    cx<T>* res = dft_run(b0, b1, P, lt, a.g.tpu);
    cx<T>* nb = (res == b0) ? b1 : b0;
    for (int k = lt; k < ny; k += a.g.tpu) {
        cx<T> c = {T(0), T(0)};
        if (!passthrough(k, P)) {
            c = get_forward(res, k, P);
            c.x *= va ? a.muinv[size_t(k) * nx + ja] : T(0);
            c.y *= vb ? a.muinv[size_t(k) * nx + jb] : T(0);
        }
        put_inverse(nb, k, c, P);
    }
    dft_pad(nb, P, lt, a.g.tpu);
    __syncthreads();
    cx<T>* res2 = dft_run(nb, res, P, lt, a.g.tpu);
    for (int t = lt; t < ny; t += a.g.tpu) {
        if (passthrough(t, P)) continue;
        const cx<T> o = get_inverse(res2, t, P);
        if (va) a.dst[size_t(t) * nx + ja] = o.x;
        if (vb) a.dst[size_t(t) * nx + jb] = o.y;
    }
}

// Diagonal / identity preconditioner iteration tail (no transform):
// convergence test of the previous residual, then x += a p, r -= a q,
// z = dinv o r (or r), ||r||^2 and <r,z> partials.
template <typename T>
__global__ void k_diag_update(int n, T* x, T* r, const T* p, const T* q, const T* dinv, T* z,
                              const double* pq_part, int n_pq, const double* rz_part, int n_rz,
                              double* rr_out, double* rz_out, PcgState* st, int iter, int do_update,
                              int check, const double* rr_in, int n_rr_in) {
    __shared__ double red[17];
    if (st->done) return;
    if (check) {
        const double rn = sqrt(sum_partials(rr_in, n_rr_in, red));
        if (iter == 0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                st->r0norm = rn;
                st->relres = rn > 0.0 ? 1.0 : 0.0;
                if (rn == 0.0) {
                    st->done = 1;
                    st->iters = 0;
                }
            }
            if (rn == 0.0) return;
        } else {
            const double r0 = st->r0norm;
            if (blockIdx.x == 0 && threadIdx.x == 0) st->relres = rn / r0;
            if (rn < st->tol * r0) {
                if (blockIdx.x == 0 && threadIdx.x == 0) {
                    st->done = 1;
                    st->iters = iter - 1;
                }
                return;
            }
        }
    }
    T step = T(0);
    if (do_update) {
        const double g = sum_partials(pq_part, n_pq, red);
        const double rz = sum_partials(rz_part, n_rz, red);
        if (!(g > 0.0)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                st->done = 2;
                st->iters = iter - 1;
            }
            return;
        }
        step = T(rz / g);
    }
    double prr = 0.0, prz = 0.0;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        T rv = r[k];
        if (do_update) {
            x[k] += step * p[k];
            rv -= step * q[k];
            r[k] = rv;
        }
        const T zv = dinv ? rv * dinv[k] : rv;
        z[k] = zv;
        prr += double(rv) * double(rv);
        prz += double(rv) * double(zv);
    }
    const double s1 = block_sum(prr, red);
    const double s2 = block_sum(prz, red);
    if (threadIdx.x == 0) {
        rr_out[blockIdx.x] = s1;
        rz_out[blockIdx.x] = s2;
    }
}

// ------------------------------------------------------------------------
// Per-step setup
// ------------------------------------------------------------------------
template <typename T>
__global__ void k_kappa(int ny, int nx, const T* __restrict__ u, double alpha, double beta, int variant,
                        T* kap, double* kapd, T* s_apply, double* s_mu, double* Dd) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= nx) return;
    const double b2 = beta * beta;
    auto U = [&](int ii, int jj) { return double(u[size_t(ii) * nx + jj]); };
    auto K = [&](int ii, int jj) {
        const double c = U(ii, jj);
        const double dx = (ii < ny - 1) ? U(ii + 1, jj) - c : 0.0;
        const double dy = (jj < nx - 1) ? U(ii, jj + 1) - c : 0.0;
        return 1.0 / sqrt(dx * dx + dy * dy + b2);
    };
    const double kc = K(i, j);
    double dl = kc * (double(i < ny - 1) + double(j < nx - 1));
    if (i > 0) dl += K(i - 1, j);
    if (j > 0) dl += K(i, j - 1);
    const double D = 1.0 + alpha * dl;
    const double s = 1.0 / sqrt(D);
    const size_t g = size_t(i) * nx + j;
    kap[g] = T(kc);
    kapd[g] = kc;
    Dd[g] = D;
    // variant: 0 none, 1 diag, 2 X, 3 D_X, 4 X_D
    if (variant == 1) s_apply[g] = T(1.0 / D);
    else if (variant == 2) s_apply[g] = T(1);
    else s_apply[g] = T(s);
    s_mu[g] = (variant == 4) ? s : 1.0;
}

__global__ void k_gemm_operands(int ny, int nx, const double* __restrict__ kap, const double* __restrict__ s,
                                double* A1, double* A2, double* A3, double* B1, double* B2, double* B3) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= nx) return;
    const size_t g = size_t(i) * nx + j;
    const double k = kap[g], sc = s[g];
    const double sd = (i < ny - 1) ? s[g + nx] : 0.0;
    const double sr = (j < nx - 1) ? s[g + 1] : 0.0;
    A1[g] = k * sd * sd;
    A2[g] = k * sd * sc;
    A3[g] = (i < ny - 1) ? k * sc * sc : 0.0;
    B1[g] = k * sr * sr;
    B2[g] = k * sr * sc;
    B3[g] = (j < nx - 1) ? k * sc * sc : 0.0;
}

// C = sum_t coef_t op(A_t) B_t, FP64, 64x64 tiles, 4x4 outputs per thread.
constexpr int kGT = 64, kGK = 16;
__global__ void __launch_bounds__(256) k_gemm(const GemmProblem* probs) {
    __shared__ double As[kGK][kGT + 1];
    __shared__ double Bs[kGK][kGT + 1];
    const GemmProblem& pb = probs[blockIdx.z];
    const int M = pb.M, N = pb.N, K = pb.K;
    if (int(blockIdx.y) * kGT >= M || int(blockIdx.x) * kGT >= N) return;
    const int tid = threadIdx.x;
    const int tm = tid / 16, tn = tid % 16;
    const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int term = 0; term < pb.nterms; ++term) {
        const double* A = pb.t[term].A;
        const double* B = pb.t[term].B;
        const double cf = pb.t[term].coef;
        for (int k0 = 0; k0 < K; k0 += kGK) {
            for (int e = tid; e < kGK * kGT; e += 256) {
                int kk, mm;
                double v = 0.0;
                if (pb.transA) {  // A stored K x M: op(A)[m][k] = A[k][m]
                    kk = e / kGT;
                    mm = e % kGT;
                    if (k0 + kk < K && m0 + mm < M) v = A[size_t(k0 + kk) * M + m0 + mm];
                } else {          // A stored M x K
                    mm = e / kGK;
                    kk = e % kGK;
                    if (k0 + kk < K && m0 + mm < M) v = A[size_t(m0 + mm) * K + k0 + kk];
                }
                As[kk][mm] = cf * v;
                const int bk = e / kGT, bn = e % kGT;
                Bs[bk][bn] = (k0 + bk < K && n0 + bn < N) ? B[size_t(k0 + bk) * N + n0 + bn] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < kGK; ++kk) {
                double av[4], bv[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) av[a] = As[kk][tm + 16 * a];
#pragma unroll
                for (int b = 0; b < 4; ++b) bv[b] = Bs[kk][tn + 16 * b];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int m = m0 + tm + 16 * a, n = n0 + tn + 16 * b;
            if (m < M && n < N) pb.C[size_t(m) * N + n] = acc[a][b];
        }
}

template <typename T>
__global__ void k_mu(int n, const double* lamh2, const double* lamx, const double* lamy, const double* lamd,
                     int use_lamd, double alpha, double* mu, T* muinv) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double h2 = lamh2[k];
    if (use_lamd) h2 *= lamd[k] * lamd[k];
    const double m = h2 + alpha * (lamx[k] + lamy[k]);
    mu[k] = m;
    muinv[k] = T(1.0 / m);
}

template <typename T>
__global__ void k_fpchange(int n, const T* x, const T* u, double* part) {
    __shared__ double red[17];
    double a = 0.0, b = 0.0;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const double xv = x[k], d = xv - double(u[k]);
        a += d * d;
        b += xv * xv;
    }
    const double s1 = block_sum(a, red);
    const double s2 = block_sum(b, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s1;
        part[2 * blockIdx.x + 1] = s2;
    }
}

__global__ void k_finalize(PcgState* st, const double* rr_part, int n_rr, const double* fp_part, int n_fp,
                           int max_iter) {
    __shared__ double red[17];
    const double rr = sum_partials(rr_part, n_rr, red);
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < n_fp; k += blockDim.x) {
        a += fp_part[2 * k];
        b += fp_part[2 * k + 1];
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    if (threadIdx.x == 0) {
        if (st->done == 0) {
            st->iters = max_iter;
            st->relres = st->r0norm > 0.0 ? sqrt(rr) / st->r0norm : 0.0;
        }
        st->fp_change = sqrt(a) / fmax(sqrt(b), 1e-300);
    }
}

__global__ void k_init_state(PcgState* st, double tol) {
    st->r0norm = 0.0;
    st->tol = tol;
    st->relres = 0.0;
    st->fp_change = 0.0;
    st->done = 0;
    st->iters = 0;
}

template <typename T>
__global__ void k_cast_double(int n, const T* src, double* dst) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = double(src[k]);
}

}  // namespace

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
int band_blocks(int ny, int nx, int ty) {
    return ((nx + kBandTX - 1) / kBandTX) * ((ny + ty - 1) / ty);
}

template <typename TX, typename TS, typename T, typename TY>
size_t band_lds_bytes(const BandArgsT<TX, TS, T, TY>& a, int ty) {
    const bool sten_tile = a.kap != nullptr && a.S == nullptr;
    const int hy = std::max(a.wy, sten_tile ? 1 : 0), hx = std::max(a.wx, sten_tile ? 1 : 0);
    size_t elems = size_t(ty + 2 * hy) * (kBandTX + 2 * hx) + size_t(ty + 2 * a.wy) * kBandTX +
                   size_t(a.nterms) * kBandTX * (2 * a.wx + 1) + size_t(a.nterms) * ty * (2 * a.wy + 1);
    if (a.kap != nullptr && a.S != nullptr) elems += size_t(ty + 2) * (kBandTX + 2);
    return elems * sizeof(T);
}

template <typename TX, typename TS, typename T, typename TY>
hipError_t launch_band(const BandArgsT<TX, TS, T, TY>& a0, int ty, hipStream_t s, int* nblocks_out) {
    if (ty != 8 && ty != 16) return hipErrorInvalidValue;
    BandArgsT<TX, TS, T, TY> a = a0;
    a.tile_y = ty;
    const size_t lds = band_lds_bytes(a, ty);
    dim3 grid((a.nx + kBandTX - 1) / kBandTX, (a.ny + ty - 1) / ty);
    if (nblocks_out) *nblocks_out = grid.x * grid.y;
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_band<TX, TS, T, TY>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    hipLaunchKernelGGL((k_band<TX, TS, T, TY>), grid, dim3(kBandThreads), lds, s, a);
    return hipGetLastError();
}

template <typename T>
LineGeom line_geom(int lines, int M) {
    LineGeom g;
    g.units = (lines + 1) / 2;
    g.tpu = std::min(256, std::max(64, M / 8));
    const size_t per_unit = size_t(2) * M * sizeof(cx<T>);
    int upb = 256 / g.tpu;
    while (upb > 1 && per_unit * upb > 64 * 1024) upb >>= 1;
    g.upb = std::min(upb, g.units);
    g.blocks = (g.units + g.upb - 1) / g.upb;
    g.lds = per_unit * g.upb;
    return g;
}

template <typename T>
hipError_t launch_rowpass(const RowPassArgs<T>& a, hipStream_t s) {
    if (a.g.lds > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rowpass<T>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(a.g.lds));
    hipLaunchKernelGGL(k_rowpass<T>, dim3(a.g.blocks), dim3(a.g.upb * a.g.tpu), a.g.lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_colpass(const ColPassArgs<T>& a, hipStream_t s) {
    if (a.g.lds > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_colpass<T>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(a.g.lds));
    hipLaunchKernelGGL(k_colpass<T>, dim3(a.g.blocks), dim3(a.g.upb * a.g.tpu), a.g.lds, s, a);
    return hipGetLastError();
}

static int elem_blocks(int n, int threads, int cap) {
    return std::max(1, std::min(cap, (n + threads - 1) / threads));
}

template <typename T>
hipError_t launch_diag_update(int n, T* x, T* r, const T* p, const T* q, const T* dinv, T* z,
                              const double* pq_part, int n_pq, const double* rz_part, int n_rz,
                              double* rr_out, double* rz_out, PcgState* st, int iter, int do_update,
                              int check, const double* rr_in, int n_rr_in, int* nblocks, hipStream_t s) {
    const int nb = elem_blocks(n, 256, 1024);
    if (nblocks) *nblocks = nb;
    hipLaunchKernelGGL(k_diag_update<T>, dim3(nb), dim3(256), 0, s, n, x, r, p, q, dinv, z, pq_part, n_pq,
                       rz_part, n_rz, rr_out, rz_out, st, iter, do_update, check, rr_in, n_rr_in);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_kappa(int ny, int nx, const T* u, double alpha, double beta, int variant, T* kap,
                        double* kapd, T* s_apply, double* s_mu, double* Dd, hipStream_t s) {
    dim3 grid((nx + 255) / 256, ny);
    hipLaunchKernelGGL(k_kappa<T>, grid, dim3(256), 0, s, ny, nx, u, alpha, beta, variant, kap, kapd, s_apply,
                       s_mu, Dd);
    return hipGetLastError();
}

hipError_t launch_gemm_operands(int ny, int nx, const double* kapd, const double* s_mu, double* A1,
                                double* A2, double* A3, double* B1, double* B2, double* B3, hipStream_t s) {
    dim3 grid((nx + 255) / 256, ny);
    hipLaunchKernelGGL(k_gemm_operands, grid, dim3(256), 0, s, ny, nx, kapd, s_mu, A1, A2, A3, B1, B2, B3);
    return hipGetLastError();
}

hipError_t launch_gemm(const GemmProblem* probs_dev, int nprob, int maxM, int maxN, hipStream_t s) {
    dim3 grid((maxN + kGT - 1) / kGT, (maxM + kGT - 1) / kGT, nprob);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, probs_dev);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mu(int n, const double* lamh2, const double* lamx, const double* lamy, const double* lamd,
                     int use_lamd, double alpha, double* mu, T* muinv, hipStream_t s) {
    hipLaunchKernelGGL(k_mu<T>, dim3((n + 255) / 256), dim3(256), 0, s, n, lamh2, lamx, lamy, lamd, use_lamd,
                       alpha, mu, muinv);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fpchange(int n, const T* x, const T* u, double* part, int* nblocks, hipStream_t s) {
    const int nb = elem_blocks(n, 256, 512);
    *nblocks = nb;
    hipLaunchKernelGGL(k_fpchange<T>, dim3(nb), dim3(256), 0, s, n, x, u, part);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_finalize(PcgState* st, const double* rr_part, int n_rr, const double* fp_part, int n_fp,
                           int max_iter, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, st, rr_part, n_rr, fp_part, n_fp, max_iter);
    return hipGetLastError();
}

hipError_t launch_init_state(PcgState* st, double tol, hipStream_t s) {
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, st, tol);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cast_to_double(int n, const T* src, double* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_cast_double<T>, dim3((n + 255) / 256), dim3(256), 0, s, n, src, dst);
    return hipGetLastError();
}

#define TVD_INSTANTIATE(T)                                                                                    \
    template hipError_t launch_band<T, T, T, T>(const BandArgs<T>&, int, hipStream_t, int*);                  \
    template size_t band_lds_bytes<T, T, T, T>(const BandArgs<T>&, int);                                      \
    template LineGeom line_geom<T>(int, int);                                                                 \
    template hipError_t launch_rowpass<T>(const RowPassArgs<T>&, hipStream_t);                                \
    template hipError_t launch_colpass<T>(const ColPassArgs<T>&, hipStream_t);                                \
    template hipError_t launch_diag_update<T>(int, T*, T*, const T*, const T*, const T*, T*, const double*,   \
                                              int, const double*, int, double*, double*, PcgState*, int, int, \
                                              int, const double*, int, int*, hipStream_t);                    \
    template hipError_t launch_kappa<T>(int, int, const T*, double, double, int, T*, double*, T*, double*,    \
                                        double*, hipStream_t);                                                \
    template hipError_t launch_mu<T>(int, const double*, const double*, const double*, const double*, int,    \
                                     double, double*, T*, hipStream_t);                                       \
    template hipError_t launch_fpchange<T>(int, const T*, const T*, double*, int*, hipStream_t);              \
    template hipError_t launch_finalize<T>(PcgState*, const double*, int, const double*, int, int,            \
                                           hipStream_t);                                                      \
    template hipError_t launch_cast_to_double<T>(int, const T*, double*, hipStream_t);

TVD_INSTANTIATE(float)
TVD_INSTANTIATE(double)

// Mixed-precision band operators of the FP32 path: FP64 coefficients and
// accumulation for the per-step residual b - A u^k and for b = H^T v.
#define TVD_INSTANTIATE_BAND(TX, TS, TA, TY)                                                                  \
    template hipError_t launch_band<TX, TS, TA, TY>(const BandArgsT<TX, TS, TA, TY>&, int, hipStream_t, int*); \
    template size_t band_lds_bytes<TX, TS, TA, TY>(const BandArgsT<TX, TS, TA, TY>&, int);

TVD_INSTANTIATE_BAND(float, float, double, float)
TVD_INSTANTIATE_BAND(float, float, double, double)
TVD_INSTANTIATE_BAND(double, float, double, float)

}  // namespace tvd

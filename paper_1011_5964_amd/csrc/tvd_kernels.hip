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

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

namespace tvd {

// Kernel timing: when a pair of events is armed, the next launch carries
// them on its own dispatch (start and end of that kernel's execution), so
// the measured time has no marker packets around it.
namespace {
thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;
thread_local bool t_ev_used = false;

template <typename F, typename... Args>
void tvd_launch(F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, Args... args) {
    if (t_ev_start) {
        hipExtLaunchKernelGGL(kernel, grid, block, std::uint32_t(lds), s, t_ev_start, t_ev_stop, 0u, args...);
        t_ev_start = t_ev_stop = nullptr;
        t_ev_used = true;
    } else {
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
    }
}
}  // namespace

void arm_kernel_events(hipEvent_t start, hipEvent_t stop) {
    t_ev_start = start;
    t_ev_stop = stop;
    t_ev_used = false;
}

bool disarm_kernel_events() {
    const bool used = t_ev_used;
    t_ev_start = t_ev_stop = nullptr;
    t_ev_used = false;
    return used;
}


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

// Global-address-space view of a device pointer.  Pointers that reach a
// kernel through memory (the batched argument tables) are generic, and loads
// through them would be flat loads, which count in both wait counters.
template <typename T>
using gmem_t = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ const gmem_t<T>* gmem(const T* p) {
    return (const gmem_t<T>*)p;
}
template <typename T>
__device__ __forceinline__ gmem_t<T>* gmem(T* p) {
    return (gmem_t<T>*)p;
}
// 16 bytes of zeros and of ones, read in place of absent epilogue operands
// (an address select instead of a branch or a select on a loaded value).
// Plain device globals, so the selected addresses stay in the global address
// space; no kernel writes them.
__device__ __align__(16) double g_nt_zeros[2] = {0.0, 0.0};
__device__ __align__(16) double g_nt_ones_d[2] = {1.0, 1.0};
__device__ __align__(16) float g_nt_ones_f[4] = {1.f, 1.f, 1.f, 1.f};
template <typename T>
__device__ __forceinline__ const T* nt_ones();
template <>
__device__ __forceinline__ const float* nt_ones<float>() {
    return g_nt_ones_f;
}
template <>
__device__ __forceinline__ const double* nt_ones<double>() {
    return g_nt_ones_d;
}

// Sum of v over the block; every thread gets the result.  red: >= 17 doubles.
__device__ __forceinline__ double block_sum(double v, double* red) {
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

// Two block sums in one pass (each summed in block_sum's order, so each
// equals block_sum of its value).  red: >= 34 doubles.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    __syncthreads();
    if (lane == 0) {
        red[w] = a;
        red[16 + w] = b;
    }
    __syncthreads();
    if (threadIdx.x < kWave) {
        double s = (threadIdx.x < nw) ? red[threadIdx.x] : 0.0;
        double t = (threadIdx.x < nw) ? red[16 + threadIdx.x] : 0.0;
        s = wave_sum(s);
        t = wave_sum(t);
        if (threadIdx.x == 0) {
            red[32] = s;
            red[33] = t;
        }
    }
    __syncthreads();
    a = red[32];
    b = red[33];
}

// Deterministic sum of n per-block partials, computed redundantly per block.
__device__ __forceinline__ double sum_partials(const double* p, int n, double* red) {
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
// Stage `count` elements into LDS with kStageBatch independent global loads in
// flight per thread (load(k) must not read memory written by store()).
constexpr int kStageBatch = 8;
template <typename V, typename Load, typename Store>
__device__ __forceinline__ void stage_lds(int count, int tid, int nthreads, Load load, Store store) {
    for (int base = tid; base < count; base += nthreads * kStageBatch) {
        V v[kStageBatch];
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int k = base + u * nthreads;
            if (k < count) v[u] = load(k);
        }
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int k = base + u * nthreads;
            if (k < count) store(k, v[u]);
        }
    }
}

template <typename TX, typename TS, typename T, typename TOut>
__device__ __forceinline__ void band_body(const BandArgsT<TX, TS, T, TOut>& a, int bx, int by, int gx) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[34];
    if (a.st && a.st->done) return;

    const int tid = threadIdx.x;
    const int tx = tid & (kBandTX - 1);
    const int ty = tid / kBandTX;            // 0..3
    const int TY = a.tile_y;
    const int i0 = by * TY;
    const int j0 = bx * kBandTX;
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
    T* Sl = byl + a.nterms * TY * by_w;                 // [(TY+2)][(TX+2)] if separate stencil input

    // p-update coefficient from the <r,z> partials of the last two iterations
    T beta = T(0);
    const bool upd = a.Z != nullptr;
    const bool use_old = upd && a.rz_old != nullptr;
    if (use_old) {
        const double rn = sum_partials(a.rz_new, a.n_rz, red);
        const double ro = sum_partials(a.rz_old, a.n_rz, red);
        beta = T(rn / ro);
    }

    // stage the input tile (zeros outside the image), p = z + beta p_old on the fly
    {
        const TX* __restrict__ Zp = a.Z;
        const TX* __restrict__ Xp = a.X;
        const TX tb = TX(beta);
        stage_lds<T>(PH * PW, tid, kBandThreads,
            [&](int k) -> T {
                const int r = k / PW, c = k - r * PW;
                int gi = i0 - hy + r, gj = j0 - hx + c;
                if (a.wrap) {  // periodic: the circulant bands read wrapped neighbours
                    gi = ((gi % ny) + ny) % ny;
                    gj = ((gj % nx) + nx) % nx;
                } else if (gi < 0 || gi >= ny || gj < 0 || gj >= nx) {
                    return T(0);
                }
                const size_t g = size_t(gi) * nx + gj;
                if (!upd) return T(Xp[g]);
                TX w = Zp[g];
                if (use_old) w += tb * Xp[g];
                return T(w);
            },
            [&](int k, T v) { P[k] = v; });
    }
    {
        const T* __restrict__ Bx = a.Bx;
        stage_lds<T>(a.nterms * kBandTX * bx_w, tid, kBandThreads,
            [&](int k) -> T {
                const int r = k / (kBandTX * bx_w);
                const int rem = k - r * kBandTX * bx_w;
                const int c = rem / bx_w, d = rem - c * bx_w;
                const int gj = j0 + c;
                return (gj < nx) ? Bx[(size_t(r) * nx + gj) * bx_w + d] : T(0);
            },
            [&](int k, T v) { bxl[k] = v; });
        const T* __restrict__ By = a.By;
        stage_lds<T>(a.nterms * TY * by_w, tid, kBandThreads,
            [&](int k) -> T {
                const int r = k / (TY * by_w);
                const int rem = k - r * TY * by_w;
                const int c = rem / by_w, d = rem - c * by_w;
                const int gi = i0 + c;
                return (gi < ny) ? By[(size_t(r) * ny + gi) * by_w + d] : T(0);
            },
            [&](int k, T v) { byl[k] = v; });
    }
    const bool sten_sep = stencil && a.S != nullptr;
    if (sten_sep) {
        const int SW = kBandTX + 2;
        const TS* __restrict__ Sp = a.S;
        stage_lds<T>((TY + 2) * SW, tid, kBandThreads,
            [&](int k) -> T {
                const int r = k / SW, c = k - r * SW;
                const int gi = i0 - 1 + r, gj = j0 - 1 + c;
                return (gi >= 0 && gi < ny && gj >= 0 && gj < nx) ? T(Sp[size_t(gi) * nx + gj]) : T(0);
            },
            [&](int k, T v) { Sl[k] = v; });
    }
    __syncthreads();
    if (upd) {  // publish the updated direction of this tile (from LDS)
        for (int r = ty; r < TY; r += 4) {
            const int gi = i0 + r, gj = j0 + tx;
            if (gi < ny && gj < nx) a.Xnew[size_t(gi) * nx + gj] = TX(P[(hy + r) * PW + hx + tx]);
        }
    }

    T acc[kBandTYMax / 4];
#pragma unroll
    for (int k = 0; k < kBandTYMax / 4; ++k) acc[k] = T(0);
    const int nacc = TY / 4;

    // rows of tmp handled by this thread-row: a contiguous block, 8 at a time,
    // so each band coefficient read from LDS serves 8 multiply-adds
    const int rpt = (TH + 3) / 4;
    const int rlo = ty * rpt, rhi = min(TH, rlo + rpt);
    constexpr int kRB = 8;
    for (int term = 0; term < a.nterms; ++term) {
        const T* bxr = bxl + (term * kBandTX + tx) * bx_w;
        for (int r0 = rlo; r0 < rhi; r0 += kRB) {
            T sacc[kRB];
#pragma unroll
            for (int u = 0; u < kRB; ++u) sacc[u] = T(0);
            const T* pbase = P + (r0 + hy - a.wy) * PW + (hx - a.wx) + tx;
            const int nr = min(kRB, rhi - r0);
            if (nr == kRB) {
                for (int d = 0; d < bx_w; ++d) {
                    const T c = bxr[d];
#pragma unroll
                    for (int u = 0; u < kRB; ++u) sacc[u] += c * pbase[u * PW + d];
                }
            } else {
                for (int d = 0; d < bx_w; ++d) {
                    const T c = bxr[d];
#pragma unroll
                    for (int u = 0; u < kRB; ++u)
                        if (u < nr) sacc[u] += c * pbase[u * PW + d];
                }
            }
#pragma unroll
            for (int u = 0; u < kRB; ++u)
                if (u < nr) tmp[(r0 + u) * kBandTX + tx] = sacc[u];
        }
        __syncthreads();
        // column pass: wave-uniform coefficients, 4 independent partial sums
#pragma unroll
        for (int k = 0; k < kBandTYMax / 4; ++k) {
            if (k >= nacc) break;
            const int ti = ty + 4 * k;
            const T* byr = byl + (term * TY + ti) * by_w;
            const T* tcol = tmp + ti * kBandTX + tx;
            T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
            int d = 0;
            for (; d + 4 <= by_w; d += 4) {
                s0 += byr[d] * tcol[d * kBandTX];
                s1 += byr[d + 1] * tcol[(d + 1) * kBandTX];
                s2 += byr[d + 2] * tcol[(d + 2) * kBandTX];
                s3 += byr[d + 3] * tcol[(d + 3) * kBandTX];
            }
            for (; d < by_w; ++d) s0 += byr[d] * tcol[d * kBandTX];
            acc[k] += (s0 + s1) + (s2 + s3);
        }
        __syncthreads();
    }

    double dot = 0.0, dot2 = 0.0;
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
            T lp = T(0);
            if (a.cst) {  // per-pixel stencil coefficients (anti-reflective L)
                const T* c4 = a.cst;
                const size_t N = size_t(ny) * nx;
                if (gi > 0) lp += c4[g] * (cen - up);
                if (gi < ny - 1) lp += c4[N + g] * (cen - dn);
                if (gj > 0) lp += c4[2 * N + g] * (cen - lf);
                if (gj < nx - 1) lp += c4[3 * N + g] * (cen - rt);
            } else {
                const T kc = a.kap[g];
                if (gi > 0) lp += a.kap[g - nx] * (cen - up);
                if (gi < ny - 1) lp += kc * (cen - dn);
                if (gj > 0) lp += a.kap[g - 1] * (cen - lf);
                if (gj < nx - 1) lp += kc * (cen - rt);
            }
            res += T(a.alpha) * lp;
        } else if (a.dotmode == 1) {
            cen = P[(hy + ti) * PW + hx + tx];
        }
        if (a.Bvec) res = a.Bvec[g] - res;
        const TOut out = TOut(res);
        a.Y[g] = out;
        if (a.dotmode == 1) dot += double(cen) * double(out);
        else if (a.dotmode == 2) dot += double(out) * double(out);
        else if (a.dotmode == 3) {
            dot += double(a.W[g]) * double(out);
            dot2 += double(out) * double(out);
        }
    }
    if (a.dotmode == 3) {
        block_sum2(dot, dot2, red);
        if (tid == 0) {
            a.dot_part[by * gx + bx] = dot;
            if (a.dot_part2) a.dot_part2[by * gx + bx] = dot2;
        }
    } else if (a.dotmode) {
        const double s = block_sum(dot, red);
        if (tid == 0) a.dot_part[by * gx + bx] = s;
    }
}

template <typename TX, typename TS, typename T, typename TOut>
__global__ void __launch_bounds__(kBandThreads) k_band(BandArgsT<TX, TS, T, TOut> a) {
    band_body(a, blockIdx.x, blockIdx.y, gridDim.x);
}

// Batched launch: image blockIdx.z, its own grid (bgx, bgy) inside the launch grid.
template <typename TX, typename TS, typename T, typename TOut>
__global__ void __launch_bounds__(kBandThreads) k_band_b(const BandArgsT<TX, TS, T, TOut>* __restrict__ as) {
    const BandArgsT<TX, TS, T, TOut> a = as[blockIdx.z];
    if (int(blockIdx.x) >= a.bgx || int(blockIdx.y) >= a.bgy) return;
    band_body(a, blockIdx.x, blockIdx.y, a.bgx);
}

// ------------------------------------------------------------------------
// Line transforms in LDS: two real lines packed as one complex sequence.
// ------------------------------------------------------------------------

// LDS slot of sequence element i: one pad entry every 8 elements keeps the
// stride-8 writes of the first radix-8 stages free of bank conflicts.
__device__ __forceinline__ int pidx(int i) { return i + (i >> 3); }
__host__ __device__ constexpr int padded_len(int M) { return M + (M >> 3); }

// LDS entries reserved for a table blob of `len` complex entries: whole
// 1 KB wave chunks of the direct global-to-LDS copy.
template <typename T>
__host__ __device__ constexpr int lds_table_len(int len) {
    return len == 0 ? 0 : ((len * int(sizeof(cx<T>)) + 1023) / 1024) * (1024 / int(sizeof(cx<T>)));
}

// In-register DFTs out[k] = sum_r a[r] exp(-2 pi i r k / R), R = 2, 4, 8.
template <typename T>
__device__ __forceinline__ void dft2(cx<T>& a0, cx<T>& a1) {
    const cx<T> t = a0;
    a0 = {t.x + a1.x, t.y + a1.y};
    a1 = {t.x - a1.x, t.y - a1.y};
}
template <typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return {a.y, -a.x}; }  // times -i
template <typename T>
__device__ __forceinline__ void dft4(cx<T>* b) {
    cx<T> c0 = b[0], c1 = b[2], c2 = b[1], c3 = b[3];
    dft2(c0, c1);  // b0 +- b2
    dft2(c2, c3);  // b1 +- b3
    c3 = mul_mi(c3);
    b[0] = {c0.x + c2.x, c0.y + c2.y};
    b[2] = {c0.x - c2.x, c0.y - c2.y};
    b[1] = {c1.x + c3.x, c1.y + c3.y};
    b[3] = {c1.x - c3.x, c1.y - c3.y};
}
template <typename T>
__device__ __forceinline__ void dft8(cx<T>* a) {
    const T h = T(0.70710678118654752440084436210484903);
    cx<T> e[4] = {a[0], a[2], a[4], a[6]};
    cx<T> o[4] = {a[1], a[3], a[5], a[7]};
    dft4(e);
    dft4(o);
    // o[k] *= exp(-2 pi i k / 8)
    o[1] = {h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)};
    o[2] = mul_mi(o[2]);
    o[3] = {h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        a[k] = {e[k].x + o[k].x, e[k].y + o[k].y};
        a[k + 4] = {e[k].x - o[k].x, e[k].y - o[k].y};
    }
}

// One Stockham decimation-in-frequency stage of radix R: for the current
// sub-transform length n = M / s, element q + s(p + r m) (m = n/R) feeds
// output q + s(R p + k) with the twiddle exp(-2 pi i p k / n) = tw[p k s].
template <typename T, int R>
__device__ __forceinline__ void stockham_stage(const cx<T>* x, cx<T>* y, int M, int log2s,
                                               const cx<T>* __restrict__ tw, int lt, int tpu) {
    const int s = 1 << log2s;
    const int nb = M / R;
    for (int b = lt; b < nb; b += tpu) {
        const int p = b >> log2s, q = b & (s - 1);
        cx<T> a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = x[pidx(b + r * nb)];
        if constexpr (R == 8) dft8(a);
        else if constexpr (R == 4) dft4(a);
        else dft2(a[0], a[1]);
        const int base = q + s * R * p;
        y[pidx(base)] = a[0];
        // w^k = exp(-2 pi i p k / n) for k = 1..R-1 from the one table entry
        // w = tw[p s] (consecutive lanes read consecutive entries): products
        // of w, w^2 and w^4, at most three roundings deep
        const cx<T> w1 = tw[p * s];
        cx<T> wk[R];
        wk[1] = w1;
        if constexpr (R >= 4) {
            wk[2] = cmul(w1, w1);
            wk[3] = cmul(wk[2], w1);
        }
        if constexpr (R == 8) {
            wk[4] = cmul(wk[2], wk[2]);
            wk[5] = cmul(wk[4], w1);
            wk[6] = cmul(wk[4], wk[2]);
            wk[7] = cmul(wk[4], wk[3]);
        }
#pragma unroll
        for (int k = 1; k < R; ++k) y[pidx(base + s * k)] = cmul(a[k], wk[k]);
    }
}

// Mixed-radix Stockham FFT (forward, exp(-2 pi i/M)) of the unit's sequence,
// radix-8 stages then one radix-4 or radix-2 stage; ping-pongs between x and
// y and returns the buffer holding the result.
template <typename T>
__device__ __forceinline__ cx<T>* fft_pow2(cx<T>* x, cx<T>* y, int M, int log2M, const cx<T>* __restrict__ tw, int lt,
                           int tpu) {
    int log2s = 0;
    while (log2s < log2M) {
        const int rem = log2M - log2s;
        const int lr = rem >= 3 ? 3 : rem;
        if (lr == 3) stockham_stage<T, 8>(x, y, M, log2s, tw, lt, tpu);
        else if (lr == 2) stockham_stage<T, 4>(x, y, M, log2s, tw, lt, tpu);
        else stockham_stage<T, 2>(x, y, M, log2s, tw, lt, tpu);
        __syncthreads();
        cx<T>* t = x;
        x = y;
        y = t;
        log2s += lr;
    }
    return x;
}

// Full DFT of length L of buffer b0 (already assembled; Bluestein inputs are
// chirp-multiplied and zero padded to M).  Returns the result buffer; the
// caller reads X_k through dft_get().
template <typename T>
__device__ __forceinline__ cx<T>* dft_run(cx<T>* b0, cx<T>* b1, const AxisPlan<T>& P, int lt, int tpu) {
    cx<T>* r = fft_pow2(b0, b1, P.M, P.log2M, P.tw, lt, tpu);
    if (!P.bluestein) return r;
    cx<T>* o = (r == b0) ? b1 : b0;
    for (int k = lt; k < P.M; k += tpu) r[pidx(k)] = cconj(cmul(r[pidx(k)], P.bf[k]));
    __syncthreads();
    return fft_pow2(r, o, P.M, P.log2M, P.tw, lt, tpu);
}

template <typename T>
__device__ __forceinline__ cx<T> dft_get(const cx<T>* r, int k, const AxisPlan<T>& P) {
    if (!P.bluestein) return r[pidx(k)];
    return cmul(P.chirp[k], cconj(r[pidx(k)]));
}

template <typename T>
__device__ __forceinline__ void dft_put(cx<T>* b, int t, cx<T> v, const AxisPlan<T>& P) {
    b[pidx(t)] = P.bluestein ? cmul(v, P.chirp[t]) : v;
}

template <typename T>
__device__ __forceinline__ void dft_pad(cx<T>* b, const AxisPlan<T>& P, int lt, int tpu) {
    if (P.bluestein)
        for (int t = P.L + lt; t < P.M; t += tpu) b[pidx(t)] = {T(0), T(0)};
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

// ---- line-pass plumbing: one batched round trip of global loads ----------

// Asynchronous copy of the plan's table blob into LDS with the direct
// global-to-LDS load (each lane moves 16 bytes to wave_base + 16 * lane);
// nothing passes through registers.  The LDS region is padded to whole
// 64-chunk waves (lds_table_len), the last wave re-reads the final chunk to
// stay inside the source.  Completion: vmcnt(0) + barrier (lds_copy_wait).
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;
__device__ __forceinline__ void lds_copy_async(const void* src, void* lds, int n16) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int4* s = reinterpret_cast<const int4*>(src);
    int4* d = reinterpret_cast<int4*>(lds);
    for (int base = wave * 64; base < n16; base += nw * 64) {
        const int k = min(base + lane, n16 - 1);
        __builtin_amdgcn_global_load_lds((glb_void_t*)(s + k), (lds_void_t*)(d + base), 16, 0, 0);
    }
}
__device__ __forceinline__ void lds_copy_wait() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// Plan whose table pointers refer to the LDS copy (or stay global).
template <typename T, bool kTabLds>
__device__ __forceinline__ AxisPlan<T> lds_plan(const AxisPlan<T>& G, cx<T>* tab) {
    AxisPlan<T> P = G;
    if constexpr (kTabLds) {
        P.tw = tab;
        P.chirp = tab + G.off_chirp;
        P.bf = tab + G.off_bf;
        P.pre = tab + G.off_pre;
        P.post = tab + G.off_post;
    }
    return P;
}

// Up to 4 per-thread partial loads summed in registers (n <= 4 * nthreads
// handled in the batch; longer lists fall back to a loop).
__device__ __forceinline__ double partial_issue(const double* p, int n, int tid, int nthr) {
    if (p == nullptr) return 0.0;
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int k = tid + u * nthr;
        if (k < n) s += p[k];
    }
    for (int k = tid + 4 * nthr; k < n; k += nthr) s += p[k];
    return s;
}

constexpr int kLinePos = 2;  // positions per thread per line (n <= 2 * tpu)

// Row pass.  mode 0: (optional x,r update) then T1 = Qx (s o r) row-wise.
//            mode 1: z = s o (Qx^T T2) row-wise, <r, z> partials.
template <typename T, bool kTabLds>
__device__ __forceinline__ void rowpass_body(const RowPassArgs<T>& a, int bx) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[17];
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int ul = tid / a.g.tpu, lt = tid - ul * a.g.tpu;
    const int unit = bx * a.g.upb + ul;
    const int nx = a.nx, ny = a.ny;
    const int tpu = a.g.tpu;
    cx<T>* tab = reinterpret_cast<cx<T>*>(smem_raw);
    const int tab_len = kTabLds ? a.plan.blob_len : 0;
    const int Mp = padded_len(a.plan.M);
    cx<T>* b0 = tab + lds_table_len<T>(tab_len) + size_t(ul) * 2 * Mp;
    cx<T>* b1 = b0 + Mp;
    T* xb_lds = reinterpret_cast<T*>(tab + lds_table_len<T>(tab_len) + size_t(a.g.upb) * 2 * Mp);
    const int ia = 2 * unit, ib = 2 * unit + 1;
    const bool va = ia < ny, vb = ib < ny;
    const size_t ga = size_t(ia) * nx, gb = size_t(ib) * nx;
    const bool upd = a.mode == 0 && a.do_update;

    // ---- one batch of global loads ----
    const int n16 = tab_len * int(sizeof(cx<T>)) / 16;
    if (kTabLds) lds_copy_async(a.plan.blob, tab, n16);
    if (a.mode == 1 && a.wout) lds_copy_async(a.xband, xb_lds, a.xband_len * int(sizeof(T)) / 16);
    const int done = a.st->done;
    const double pq = upd ? partial_issue(a.pq_part, a.n_pq, tid, nthr) : 0.0;
    const double rzp = upd ? partial_issue(a.rz_part, a.n_rz, tid, nthr) : 0.0;
    T ra[kLinePos], rb[kLinePos], xa[kLinePos], xb[kLinePos], pa[kLinePos], pb[kLinePos], qa[kLinePos],
        qb[kLinePos], sa[kLinePos], sb[kLinePos];
    const T* src = a.mode == 0 ? a.r : a.src;
#pragma unroll
    for (int c = 0; c < kLinePos; ++c) {
        const int t = lt + c * tpu;
        const bool in = t < nx;
        ra[c] = (in && va) ? src[ga + t] : T(0);
        rb[c] = (in && vb) ? src[gb + t] : T(0);
        sa[c] = (in && va && a.s) ? a.s[ga + t] : T(1);
        sb[c] = (in && vb && a.s) ? a.s[gb + t] : T(1);
        if (upd) {
            xa[c] = (in && va) ? a.x[ga + t] : T(0);
            xb[c] = (in && vb) ? a.x[gb + t] : T(0);
            pa[c] = (in && va) ? a.p[ga + t] : T(0);
            pb[c] = (in && vb) ? a.p[gb + t] : T(0);
            qa[c] = (in && va) ? a.q[ga + t] : T(0);
            qb[c] = (in && vb) ? a.q[gb + t] : T(0);
        }
        if (a.mode == 1) {  // r for the <r, z> dot
            xa[c] = (in && va) ? a.r[ga + t] : T(0);
            xb[c] = (in && vb) ? a.r[gb + t] : T(0);
        }
    }
    // T_n: the two end values of each line (mode 0: of s o r), whose linear
    // interpolant the interior loses before S^ (mode 0) or gains after it
    T e0a = T(0), e1a = T(0), e0b = T(0), e1b = T(0);
    if (a.ramp) {
        const bool sm0 = a.mode == 0 && a.s;
        if (va) {
            e0a = src[ga] * (sm0 ? a.s[ga] : T(1));
            e1a = src[ga + nx - 1] * (sm0 ? a.s[ga + nx - 1] : T(1));
        }
        if (vb) {
            e0b = src[gb] * (sm0 ? a.s[gb] : T(1));
            e1b = src[gb + nx - 1] * (sm0 ? a.s[gb + nx - 1] : T(1));
        }
    }
    const T inv_span = T(1) / T(nx - 1);
    lds_copy_wait();
    if (done) return;
    const AxisPlan<T> P = lds_plan<T, kTabLds>(a.plan, tab);

    double part = 0.0;
    if (a.mode == 0) {
        T step = T(0);
        if (upd) {
            const double g = block_sum(pq, red);
            const double rz = block_sum(rzp, red);
            if (!(g > 0.0)) {  // curvature <= 0 (or NaN): stop, keep x_{i-1}
                if (bx == 0 && tid == 0) {
                    a.st->done = 2;
                    a.st->iters = a.iter - 1;
                }
                return;
            }
            step = T(rz / g);
        }
#pragma unroll
        for (int c = 0; c < kLinePos; ++c) {
            const int t = lt + c * tpu;
            if (t >= nx) continue;
            T va_ = ra[c], vb_ = rb[c];
            if (upd) {
                va_ -= step * qa[c];
                vb_ -= step * qb[c];
                if (va) {
                    a.x[ga + t] = xa[c] + step * pa[c];
                    a.r[ga + t] = va_;
                    part += double(va_) * double(va_);
                }
                if (vb) {
                    a.x[gb + t] = xb[c] + step * pb[c];
                    a.r[gb + t] = vb_;
                    part += double(vb_) * double(vb_);
                }
            }
            va_ *= sa[c];
            vb_ *= sb[c];
            if (passthrough(t, P)) {
                if (va) a.dst[ga + t] = va_;
                if (vb) a.dst[gb + t] = vb_;
            } else if (a.ramp) {
                const T f = T(t) * inv_span;
                va_ -= (T(1) - f) * e0a + f * e1a;
                vb_ -= (T(1) - f) * e0b + f * e1b;
            }
            put_forward(b0, t, cx<T>{va_, vb_}, P);
        }
        dft_pad(b0, P, lt, tpu);
        __syncthreads();
        cx<T>* res = dft_run(b0, b1, P, lt, tpu);
        for (int k = lt; k < nx; k += tpu) {
            if (passthrough(k, P)) continue;
            const cx<T> o = get_forward(res, k, P);
            if (va) a.dst[ga + k] = o.x;
            if (vb) a.dst[gb + k] = o.y;
        }
        if (upd) {
            const double sm = block_sum(part, red);
            if (tid == 0) a.part_out[bx] = sm;
        }
    } else {
        T zpa[kLinePos], zpb[kLinePos];
#pragma unroll
        for (int c = 0; c < kLinePos; ++c) {
            const int k = lt + c * tpu;
            zpa[c] = zpb[c] = T(0);
            if (k >= nx) continue;
            if (passthrough(k, P)) {
                const T za = sa[c] * ra[c], zb = sb[c] * rb[c];
                zpa[c] = za;
                zpb[c] = zb;
                if (va) {
                    a.dst[ga + k] = za;
                    part += double(xa[c]) * double(za);
                }
                if (vb) {
                    a.dst[gb + k] = zb;
                    part += double(xb[c]) * double(zb);
                }
            }
            put_inverse(b0, k, cx<T>{ra[c], rb[c]}, P);
        }
        dft_pad(b0, P, lt, tpu);
        __syncthreads();
        cx<T>* res = dft_run(b0, b1, P, lt, tpu);
        cx<T>* zc = (res == b0) ? b1 : b0;  // free buffer: z of both lines for the x-pass
#pragma unroll
        for (int c = 0; c < kLinePos; ++c) {
            const int t = lt + c * tpu;
            if (t >= nx) continue;
            T za = zpa[c], zb = zpb[c];
            if (!passthrough(t, P)) {
                cx<T> o = get_inverse(res, t, P);
                if (a.ramp) {
                    const T f = T(t) * inv_span;
                    o.x += (T(1) - f) * e0a + f * e1a;
                    o.y += (T(1) - f) * e0b + f * e1b;
                }
                za = sa[c] * o.x;
                zb = sb[c] * o.y;
                if (va) {
                    a.dst[ga + t] = za;
                    part += double(xa[c]) * double(za);
                }
                if (vb) {
                    a.dst[gb + t] = zb;
                    part += double(xb[c]) * double(zb);
                }
            }
            if (a.wout) zc[t] = cx<T>{za, zb};
        }
        if (a.wout) {
            // w = (I (x) K_x) z on both lines: Toeplitz row in the interior,
            // stored rows near the edges; taps outside the line have zero
            // coefficients (indices clamped only to stay inside the buffer).
            const int bw = 2 * a.kw + 1;
            __syncthreads();
            lds_copy_wait();
#pragma unroll
            for (int c = 0; c < kLinePos; ++c) {
                const int t = lt + c * tpu;
                if (t >= nx) continue;
                const int rr = t < a.klo ? 1 + t : (t >= a.khi ? 1 + a.klo + (t - a.khi) : 0);
                const T* coef = xb_lds + rr * bw;
                T sa_ = T(0), sb_ = T(0);
                for (int d = 0; d < bw; ++d) {
                    const int idx = min(max(t + d - a.kw, 0), nx - 1);
                    const cx<T> zv = zc[idx];
                    sa_ += coef[d] * zv.x;
                    sb_ += coef[d] * zv.y;
                }
                if (va) a.wout[ga + t] = sa_;
                if (vb) a.wout[gb + t] = sb_;
            }
        }
        const double sm = block_sum(part, red);
        if (tid == 0) a.part_out[bx] = sm;
    }
}

template <typename T, bool kTabLds>
__global__ void k_rowpass(RowPassArgs<T> a) {
    rowpass_body<T, kTabLds>(a, blockIdx.x);
}

template <typename T, bool kTabLds>
__global__ void k_rowpass_b(const RowPassArgs<T>* __restrict__ as, int it) {
    RowPassArgs<T> a = as[blockIdx.z];
    if (int(blockIdx.x) >= a.g.blocks || a.st->done) return;  // converged images idle
    a.iter = it;
    rowpass_body<T, kTabLds>(a, blockIdx.x);
}

// PCG stopping test (strict ||r|| < tol ||r_0||, Section 5) from this
// thread's share rrp of the ||r||^2 partials; every block evaluates it and
// `leader` (one thread of the grid) records it.  At iteration 0 it fixes
// ||r_0|| (zero: converged in 0 iterations).  A replay cap > 0 stops after
// exactly that many iterations.  Returns true when the block must stop.
__device__ __forceinline__ bool pcg_stop_test(PcgState* st, double rrp, int iter, double r0, double tol, int cap,
                                              bool leader, double* red) {
    const double rn = sqrt(block_sum(rrp, red));
    if (iter == 0) {
        if (leader) {
            st->r0norm = rn;
            st->relres = rn > 0.0 ? 1.0 : 0.0;
            if (rn == 0.0) {
                st->done = 1;
                st->iters = 0;
            }
        }
        return rn == 0.0;
    }
    if (leader) st->relres = rn / r0;
    if (rn < tol * r0 || (cap > 0 && iter >= cap)) {
        if (leader) {
            st->done = 1;
            st->iters = iter;
        }
        return true;
    }
    return false;
}

// Block index -> work index such that the blocks the hardware places on one
// XCD (dispatch is round-robin over the 8 XCDs: block b runs on XCD b % 8)
// take one contiguous range of work: neighbouring columns and tiles then
// share that XCD's L2 instead of being fetched into all eight.  A bijection
// on [0, nb).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    constexpr int kXcd = 8;
    const int x = b % kXcd, j = b / kXcd;
    const int q = nb / kXcd, r = nb % kXcd;
    return x * q + min(x, r) + j;
}

// Block -> 32 x 32 tile (bx, by) of a gx x gy product grid.  When the grid
// splits into 4 x 2 equal sub-grids, the blocks of one XCD (b % 8) take one
// sub-grid: its L2 then fetches gy/2 row slabs of A and gx/4 of Bt instead of
// two row slabs and the whole of Bt (contiguous ranges of tiles).  Otherwise
// contiguous ranges.  A bijection on the tiles.
__device__ __forceinline__ void tile_of_block(int b, int gx, int gy, int& bx, int& by) {
    if ((gx & 3) == 0 && (gy & 1) == 0) {
        const int x = b & 7, j = b >> 3, sw = gx >> 2;
        bx = (x & 3) * sw + j % sw;
        by = (x >> 2) * (gy >> 1) + j / sw;
    } else {
        const int w = xcd_remap(b, gx * gy);
        bx = w % gx;
        by = w / gx;
    }
}

// Column pass: convergence test, forward column transform, divide by mu,
// inverse column transform.
template <typename T, bool kTabLds>
__device__ __forceinline__ void colpass_body(const ColPassArgs<T>& a, int bx) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[17];
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int ul = tid / a.g.tpu, lt = tid - ul * a.g.tpu;
    const int unit = bx * a.g.upb + ul;
    const int nx = a.nx, ny = a.ny;
    const int tpu = a.g.tpu;
    cx<T>* tab = reinterpret_cast<cx<T>*>(smem_raw);
    const int tab_len = kTabLds ? a.plan.blob_len : 0;
    const int Mp = padded_len(a.plan.M);
    cx<T>* b0 = tab + lds_table_len<T>(tab_len) + size_t(ul) * 2 * Mp;
    cx<T>* b1 = b0 + Mp;
    const int ja = 2 * unit, jb = 2 * unit + 1;
    const bool va = ja < nx, vb = jb < nx;

    // ---- one batch of global loads ----
    const int n16 = tab_len * int(sizeof(cx<T>)) / 16;
    if (kTabLds) lds_copy_async(a.plan.blob, tab, n16);
    const int done = a.st->done;
    const double r0 = a.st->r0norm;
    const double tol = a.st->tol;
    const int cap = a.st->cap;
    const double rrp = a.check ? partial_issue(a.rr_part, a.n_rr, tid, nthr) : 0.0;
    T xa[kLinePos], xb[kLinePos], ma[kLinePos], mb[kLinePos];
#pragma unroll
    for (int c = 0; c < kLinePos; ++c) {
        const int t = lt + c * tpu;
        const bool in = t < ny;
        const size_t g = size_t(t) * nx;
        xa[c] = (in && va) ? a.src[g + ja] : T(0);
        xb[c] = (in && vb) ? a.src[g + jb] : T(0);
        ma[c] = (in && va) ? a.muinv[g + ja] : T(0);
        mb[c] = (in && vb) ? a.muinv[g + jb] : T(0);
    }
    // T_n along the columns: end values and their scaled coefficients
    T x0a = T(0), x1a = T(0), x0b = T(0), x1b = T(0), c0a = T(0), c1a = T(0), c0b = T(0), c1b = T(0);
    if (a.ramp) {
        const size_t gl = size_t(ny - 1) * nx;
        if (va) {
            x0a = a.src[ja];
            x1a = a.src[gl + ja];
            c0a = x0a * a.muinv[ja];
            c1a = x1a * a.muinv[gl + ja];
        }
        if (vb) {
            x0b = a.src[jb];
            x1b = a.src[gl + jb];
            c0b = x0b * a.muinv[jb];
            c1b = x1b * a.muinv[gl + jb];
        }
    }
    const T inv_span = T(1) / T(ny - 1);
    lds_copy_wait();
    if (done) return;
    if (a.check && pcg_stop_test(a.st, rrp, a.iter, r0, tol, cap, bx == 0 && tid == 0, red)) return;
    const AxisPlan<T> P = lds_plan<T, kTabLds>(a.plan, tab);
#pragma unroll
    for (int c = 0; c < kLinePos; ++c) {
        const int t = lt + c * tpu;
        if (t >= ny) continue;
        if (passthrough(t, P)) {
            if (va) a.dst[size_t(t) * nx + ja] = xa[c] * ma[c];
            if (vb) a.dst[size_t(t) * nx + jb] = xb[c] * mb[c];
        } else if (a.ramp) {
            const T f = T(t) * inv_span;
            xa[c] -= (T(1) - f) * x0a + f * x1a;
            xb[c] -= (T(1) - f) * x0b + f * x1b;
        }
        put_forward(b0, t, cx<T>{xa[c], xb[c]}, P);
    }
    dft_pad(b0, P, lt, tpu);
    __syncthreads();
    cx<T>* res = dft_run(b0, b1, P, lt, tpu);
    cx<T>* nb = (res == b0) ? b1 : b0;
#pragma unroll
    for (int c = 0; c < kLinePos; ++c) {
        const int k = lt + c * tpu;
        if (k >= ny) continue;
        cx<T> v = {T(0), T(0)};
        if (!passthrough(k, P)) {
            v = get_forward(res, k, P);
            v.x *= ma[c];
            v.y *= mb[c];
        }
        put_inverse(nb, k, v, P);
    }
    dft_pad(nb, P, lt, tpu);
    __syncthreads();
    cx<T>* res2 = dft_run(nb, res, P, lt, tpu);
#pragma unroll
    for (int c = 0; c < kLinePos; ++c) {
        const int t = lt + c * tpu;
        if (t >= ny || passthrough(t, P)) continue;
        cx<T> o = get_inverse(res2, t, P);
        if (a.ramp) {
            const T f = T(t) * inv_span;
            o.x += (T(1) - f) * c0a + f * c1a;
            o.y += (T(1) - f) * c0b + f * c1b;
        }
        if (va) a.dst[size_t(t) * nx + ja] = o.x;
        if (vb) a.dst[size_t(t) * nx + jb] = o.y;
    }
}

template <typename T, bool kTabLds>
__global__ void k_colpass(ColPassArgs<T> a) {
    colpass_body<T, kTabLds>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, bool kTabLds>
__global__ void k_colpass_b(const ColPassArgs<T>* __restrict__ as, int it) {
    ColPassArgs<T> a = as[blockIdx.z];
    const int bx = xcd_remap(blockIdx.x, gridDim.x);
    if (bx >= a.g.blocks || a.st->done) return;
    a.iter = it;
    colpass_body<T, kTabLds>(a, bx);
}

// Column half of the fused normal operator (see YPassArgs), 64 x 16 outputs
// per block, one output per thread, all inputs in one batch of loads.
constexpr int kYTX = 64, kYTY = 16, kYThreads = kYTX * kYTY;
template <typename T>
__device__ __forceinline__ void ypass_body(const YPassArgs<T>& a, int bx, int by, int gx) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[17];
    const int tid = threadIdx.x, tx = tid & (kYTX - 1), ty = tid / kYTX;
    const int tyu = __builtin_amdgcn_readfirstlane(ty);
    const int i0 = by * kYTY, j0 = bx * kYTX;
    const int ny = a.ny, nx = a.nx, w = a.w;
    const int TH = kYTY + 2 * w;
    constexpr int PW = kYTX + 2;
    T* tt = reinterpret_cast<T*>(smem_raw);  // [TH][kYTX]  tmp_new
    T* pt = tt + TH * kYTX;                  // [kYTY + 2][PW] p_new
    const bool use_old = a.rz_old != nullptr;

    // ---- one batch of global loads ----
    const int done = a.st ? a.st->done : 0;
    const double rzn = use_old ? partial_issue(a.rz_new, a.n_rz, tid, kYThreads) : 0.0;
    const double rzo = use_old ? partial_issue(a.rz_old, a.n_rz, tid, kYThreads) : 0.0;
    constexpr int kTS = 5;  // (16 + 2*32) * 64 / 1024
    T wv[kTS], to[kTS];
#pragma unroll
    for (int k = 0; k < kTS; ++k) {
        const int e = tid + k * kYThreads;
        const int r = e / kYTX, c = e - r * kYTX;
        const int gi = i0 - w + r, gj = j0 + c;
        const bool in = e < TH * kYTX && gi >= 0 && gi < ny && gj < nx;
        const size_t g = in ? size_t(gi) * nx + gj : 0;
        wv[k] = in ? a.wv[g] : T(0);
        to[k] = (in && use_old) ? a.tmp_old[g] : T(0);
    }
    constexpr int kPS = 2;  // (16 + 2) * 66 = 1188 <= 2 * 1024
    T zv[kPS], po[kPS];
#pragma unroll
    for (int k = 0; k < kPS; ++k) {
        const int e = tid + k * kYThreads;
        const int r = e / PW, c = e - r * PW;
        const int gi = i0 - 1 + r, gj = j0 - 1 + c;
        const bool in = e < (kYTY + 2) * PW && gi >= 0 && gi < ny && gj >= 0 && gj < nx;
        const size_t g = in ? size_t(gi) * nx + gj : 0;
        zv[k] = in ? a.z[g] : T(0);
        po[k] = (in && use_old) ? a.p_old[g] : T(0);
    }
    const int gi = i0 + ty, gj = j0 + tx;
    const bool own = gi < ny && gj < nx;
    const size_t g = own ? size_t(gi) * nx + gj : 0;
    const T kc = own ? a.kap[g] : T(0);
    const T ku = (own && gi > 0) ? a.kap[g - nx] : T(0);
    const T kl = (own && gj > 0) ? a.kap[g - 1] : T(0);
    if (done) return;

    T beta = T(0);
    if (use_old) {
        const double n_ = block_sum(rzn, red);
        const double o_ = block_sum(rzo, red);
        beta = T(n_ / o_);
    }
#pragma unroll
    for (int k = 0; k < kTS; ++k) {
        const int e = tid + k * kYThreads;
        if (e < TH * kYTX) tt[e] = wv[k] + beta * to[k];
    }
#pragma unroll
    for (int k = 0; k < kPS; ++k) {
        const int e = tid + k * kYThreads;
        if (e < (kYTY + 2) * PW) pt[e] = zv[k] + beta * po[k];
    }
    __syncthreads();

    double dot = 0.0;
    if (own) {
        const T* prow = pt + (ty + 1) * PW + tx + 1;
        const T pc = prow[0];
        a.tmp_new[g] = tt[(ty + w) * kYTX + tx];
        a.p_new[g] = pc;
        const int row = min(i0 + tyu, ny - 1);  // wave-uniform band row
        const T* kyr = a.Ky + size_t(row) * (2 * w + 1);
        const T* tcol = tt + ty * kYTX + tx;
        T s0 = T(0), s1 = T(0);
        int d = 0;
        for (; d + 2 <= 2 * w + 1; d += 2) {
            s0 += kyr[d] * tcol[d * kYTX];
            s1 += kyr[d + 1] * tcol[(d + 1) * kYTX];
        }
        if (d < 2 * w + 1) s0 += kyr[d] * tcol[d * kYTX];
        T lp = T(0);
        if (gi > 0) lp += ku * (pc - prow[-PW]);
        if (gi < ny - 1) lp += kc * (pc - prow[PW]);
        if (gj > 0) lp += kl * (pc - prow[-1]);
        if (gj < nx - 1) lp += kc * (pc - prow[1]);
        const T qv = (s0 + s1) + T(a.alpha) * lp;
        a.q[g] = qv;
        dot = double(pc) * double(qv);
    }
    const double sm = block_sum(dot, red);
    if (tid == 0) a.pq_part[by * gx + bx] = sm;
}

template <typename T>
__global__ void __launch_bounds__(kYThreads) k_ypass(YPassArgs<T> a) {
    ypass_body(a, blockIdx.x, blockIdx.y, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(kYThreads) k_ypass_b(const YPassArgs<T>* __restrict__ as) {
    const YPassArgs<T> a = as[blockIdx.z];
    const int gx = (a.nx + kYTX - 1) / kYTX, gy = (a.ny + kYTY - 1) / kYTY;
    if (int(blockIdx.x) >= gx || int(blockIdx.y) >= gy || a.st->done) return;
    ypass_body(a, blockIdx.x, blockIdx.y, gx);
}

// The whole normal operator in one tile pass (no row half elsewhere):
// p = z + beta p_old over the 64 x 16 tile and a halo of the band half-widths
// on all sides (columns clamped to the image, as the row band expects; rows
// outside the image are zero), then K_y down the columns of the tile rows,
// K_x along them (Toeplitz interior row, stored edge rows), the TV stencil and
// <p, q> partials.  Both half-widths <= kYFMaxH.
constexpr int kYFMaxH = 32;
template <typename T>
__device__ __forceinline__ T band_dot(const T* __restrict__ coef, const T* v, int bw) {
    T s0 = T(0), s1 = T(0);
    int d = 0;
    for (; d + 2 <= bw; d += 2) {
        s0 += coef[d] * v[d];
        s1 += coef[d + 1] * v[d + 1];
    }
    if (d < bw) s0 += coef[d] * v[d];
    return s0 + s1;
}
constexpr int kYFRegs = ((kYTY + 2 * kYFMaxH) * (kYTX + 2 * kYFMaxH) + kYThreads - 1) / kYThreads;
// kRowPairs: the beta sums in one reduction and K_y two tile rows per
// thread (the single-image kernel; measured slower in the batched one).
// kBcg: the BiCGstab form (see YPassArgs): q = A z with the partials of
// <dotw, q> and <q, q>, no direction update.
template <typename T, bool kRowPairs, bool kBcg = false>
__device__ __forceinline__ void ypass_full_body(const YPassArgs<T>& a, int bx, int by, int gx) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[34];
    const int tid = threadIdx.x, tx = tid & (kYTX - 1), ty = tid / kYTX;
    const int i0 = by * kYTY, j0 = bx * kYTX;
    const int ny = a.ny, nx = a.nx, wy = a.w, wx = a.kw;
    const int hy = max(wy, 1), hx = max(wx, 1);
    const int TH = kYTY + 2 * hy, TW = kYTX + 2 * hx, nreg = TH * TW;
    T* pr = reinterpret_cast<T*>(smem_raw);  // [TH][TW] p_new, tile + halo
    T* ar = pr + nreg;                       // [kYTY][TW] K_y p_new
    const bool use_old = a.rz_old != nullptr;

    // ---- one batch of global loads ----
    const int done = a.st ? a.st->done : 0;
    const double rzn = use_old ? partial_issue(a.rz_new, a.n_rz, tid, kYThreads) : 0.0;
    const double rzo = use_old ? partial_issue(a.rz_old, a.n_rz, tid, kYThreads) : 0.0;
    T zv[kYFRegs], po[kYFRegs];
#pragma unroll
    for (int k = 0; k < kYFRegs; ++k) {
        const int e = tid + k * kYThreads;
        const int r = e / TW, c = e - r * TW;
        int gi = i0 - hy + r, gj = j0 - hx + c;
        if (a.wrap) {  // periodic: rows and columns of the halo wrap around
            gi = ((gi % ny) + ny) % ny;
            gj = ((gj % nx) + nx) % nx;
        } else {
            gj = min(max(gj, 0), nx - 1);
        }
        const bool in = e < nreg && gi >= 0 && gi < ny;
        const size_t g = in ? size_t(gi) * nx + gj : 0;
        zv[k] = in ? a.z[g] : T(0);
        po[k] = (in && use_old) ? a.p_old[g] : T(0);
    }
    const int gi = i0 + ty, gj = j0 + tx;
    const bool own = gi < ny && gj < nx;
    const size_t g = own ? size_t(gi) * nx + gj : 0;
    // stencil coefficients up / down / left / right: the cell diffusivity
    // (zero-Neumann L) or the per-pixel ones of the anti-reflective L
    T c_up, c_dn, c_lf, c_rt;
    if (kBcg && a.cst) {
        const size_t N = size_t(ny) * nx;
        c_up = own ? a.cst[g] : T(0);
        c_dn = own ? a.cst[N + g] : T(0);
        c_lf = own ? a.cst[2 * N + g] : T(0);
        c_rt = own ? a.cst[3 * N + g] : T(0);
    } else {
        const T kc = own ? a.kap[g] : T(0);
        c_up = (own && gi > 0) ? a.kap[g - nx] : T(0);
        c_lf = (own && gj > 0) ? a.kap[g - 1] : T(0);
        c_dn = kc;
        c_rt = kc;
    }
    T dw = T(0);
    if constexpr (kBcg) dw = own ? a.dotw[g] : T(0);
    if (done) return;

    T beta = T(0);
    if (use_old) {
        double n_ = rzn, o_ = rzo;
        if constexpr (kRowPairs) {
            block_sum2(n_, o_, red);
        } else {
            n_ = block_sum(n_, red);
            o_ = block_sum(o_, red);
        }
        beta = T(n_ / o_);
    }
#pragma unroll
    for (int k = 0; k < kYFRegs; ++k) {
        const int e = tid + k * kYThreads;
        if (e < nreg) pr[e] = zv[k] + beta * po[k];
    }
    __syncthreads();

    if constexpr (!kRowPairs) {
        // K_y: tile row ty (wave-uniform band row), every column of the region
        const int row = min(i0 + int(__builtin_amdgcn_readfirstlane(ty)), ny - 1);
        const T* kyr = a.Ky + size_t(row) * (2 * wy + 1);
        for (int c = tx; c < TW; c += kYTX) {
            const T* col = pr + (ty + hy - wy) * TW + c;
            T s0 = T(0), s1 = T(0);
            int d = 0;
            for (; d + 2 <= 2 * wy + 1; d += 2) {
                s0 += kyr[d] * col[d * TW];
                s1 += kyr[d + 1] * col[(d + 1) * TW];
            }
            if (d < 2 * wy + 1) s0 += kyr[d] * col[d * TW];
            ar[ty * TW + c] = s0 + s1;
        }
    } else {
        // K_y: each wave takes a pair of tile rows (wave-uniform band rows) and
        // half of the region's columns; a thread sums both rows of its column
        // from one pass down it (the even and odd taps of each row in separate
        // accumulators, as for a single row)
        const int wv = __builtin_amdgcn_readfirstlane(ty);
        const int r0 = 2 * (wv & 7), c = (wv >> 3) * kYTX + tx;
        const gmem_t<T>* ky0 = gmem(a.Ky) + size_t(min(i0 + r0, ny - 1)) * (2 * wy + 1);
        const gmem_t<T>* ky1 = gmem(a.Ky) + size_t(min(i0 + r0 + 1, ny - 1)) * (2 * wy + 1);
        if (c < TW) {
            const T* col = pr + (r0 + hy - wy) * TW + c;
            T e0 = T(0), o0 = T(0), e1 = T(0), o1 = T(0);
            e0 += ky0[0] * col[0];
            int d = 1;
            for (; d + 2 <= 2 * wy + 1; d += 2) {
                const T v1 = col[d * TW], v2 = col[(d + 1) * TW];
                o0 += ky0[d] * v1;
                e1 += ky1[d - 1] * v1;
                e0 += ky0[d + 1] * v2;
                o1 += ky1[d] * v2;
            }
            if (d < 2 * wy + 1) {
                const T v1 = col[d * TW];
                o0 += ky0[d] * v1;
                e1 += ky1[d - 1] * v1;
                ++d;
            }
            // row r0 + 1's last tap (its d' = 2 wy, at d = 2 wy + 1)
            const T vl = col[(2 * wy + 1) * TW];
            if ((2 * wy) & 1) o1 += ky1[2 * wy] * vl;
            else e1 += ky1[2 * wy] * vl;
            ar[r0 * TW + c] = e0 + o0;
            ar[(r0 + 1) * TW + c] = e1 + o1;
        }
    }
    __syncthreads();

    double dot = 0.0, dot2 = 0.0;
    if (own) {
        const T* prow = pr + (ty + hy) * TW + tx + hx;
        const T pc = prow[0];
        if constexpr (!kBcg) a.p_new[g] = pc;
        // K_x along the row: interior tiles use the Toeplitz row (uniform
        // coefficients), tiles that touch a stored edge row pick per column
        const int bw = 2 * wx + 1;
        const T* arow = ar + ty * TW + tx + hx - wx;
        T kxp;
        if (j0 >= a.klo && j0 + kYTX <= a.khi) {
            kxp = band_dot(a.xband, arow, bw);
        } else {
            const int rr = gj < a.klo ? 1 + gj : (gj >= a.khi ? 1 + a.klo + (gj - a.khi) : 0);
            kxp = band_dot(a.xband + size_t(rr) * bw, arow, bw);
        }
        T lp = T(0);
        if (gi > 0) lp += c_up * (pc - prow[-TW]);
        if (gi < ny - 1) lp += c_dn * (pc - prow[TW]);
        if (gj > 0) lp += c_lf * (pc - prow[-1]);
        if (gj < nx - 1) lp += c_rt * (pc - prow[1]);
        const T qv = kxp + T(a.alpha) * lp;
        a.q[g] = qv;
        if constexpr (kBcg) {
            dot = double(dw) * double(qv);
            dot2 = double(qv) * double(qv);
        } else {
            dot = double(pc) * double(qv);
        }
    }
    if constexpr (kBcg) {
        block_sum2(dot, dot2, red);
        if (tid == 0) {
            a.pq_part[by * gx + bx] = dot;
            if (a.qq_part) a.qq_part[by * gx + bx] = dot2;
        }
    } else {
        const double sm = block_sum(dot, red);
        if (tid == 0) a.pq_part[by * gx + bx] = sm;
    }
}

template <typename T>
__global__ void __launch_bounds__(kYThreads) k_ypass_full(YPassArgs<T> a) {
    ypass_full_body<T, true>(a, blockIdx.x, blockIdx.y, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(kYThreads) k_ypass_full_bcg(YPassArgs<T> a) {
    ypass_full_body<T, true, true>(a, blockIdx.x, blockIdx.y, gridDim.x);
}

// Image of block b of a compact batched grid: the last i with prefix[i] <= b.
__device__ __forceinline__ int batch_image(const int* __restrict__ prefix, int count, int b) {
    int lo = 0, hi = count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <typename T>
__global__ void __launch_bounds__(kYThreads) k_ypass_full_b(const YPassArgs<T>* __restrict__ as) {
    const YPassArgs<T> a = as[blockIdx.z];
    const int gx = (a.nx + kYTX - 1) / kYTX, gy = (a.ny + kYTY - 1) / kYTY;
    if (int(blockIdx.x) >= gx || int(blockIdx.y) >= gy || a.st->done) return;
    ypass_full_body<T, false>(a, blockIdx.x, blockIdx.y, gx);
}

// The same on a compact grid (one block per tile of each image).
template <typename T>
__global__ void __launch_bounds__(kYThreads) k_ypass_full_bc(const YPassArgs<T>* __restrict__ as,
                                                             const int* __restrict__ prefix, int count) {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int img = batch_image(prefix, count, b);
    const YPassArgs<T> a = as[img];
    if (a.st->done) return;
    const int gx = (a.nx + kYTX - 1) / kYTX;
    const int local = b - prefix[img];
    ypass_full_body<T, false>(a, local % gx, local / gx, gx);
}

// ------------------------------------------------------------------------
// Dense products on the matrix cores (MFMA 16x16x4 in FP32 and FP64; the
// FP32 64 x 64 tiles use bf16 16x16x32 on split operands, see mma_split6).
// MfmaCfg holds the FP32 / FP64 instruction and its lane layout per type.
// ------------------------------------------------------------------------
template <typename T>
struct MfmaCfg;

template <>
struct MfmaCfg<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; result r of
    // lane l is C[4 (l / 16) + r][l % 16]
    static __device__ __forceinline__ int orow(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <>
struct MfmaCfg<double> {
    // K slice and LDS strides of the multi-term setup products (k_mgemm_multi)
    static constexpr int BK = 32, SA = 33, SB = 32;
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // operands as for float; result r of lane l is C[l / 16 + 4 r][l % 16]
    static __device__ __forceinline__ int orow(int lane, int r) { return (lane >> 4) + 4 * r; }
};

// One K slice of a wave's 16 x 16 tile from the LDS copies of A (row-major,
// stride SA) and B (k-major, stride SB).
template <typename T>
__device__ __forceinline__ void mma_slice(const T* As, const T* Bs, int lane, int wr, int wc,
                                          typename MfmaCfg<T>::acc_t& acc) {
    using Cfg = MfmaCfg<T>;
    const T* as = As + (wr + (lane & 15)) * Cfg::SA + (lane >> 4);
    const T* bs = Bs + (lane >> 4) * Cfg::SB + wc + (lane & 15);
#pragma unroll
    for (int kk = 0; kk < Cfg::BK / 4; ++kk) acc = Cfg::mma(as[4 * kk], bs[4 * kk * Cfg::SB], acc);
}

// FP32 products from bf16 matrix instructions: each FP32 operand is split
// into three bf16 parts x = h + m + l (h = bf16(x), m = bf16(x - h),
// l = bf16(x - h - m), round to nearest; both differences are exact in FP32)
// and the product is the sum of the six part products of order 2^-16 |x y|
// and above (hh, hm, mh, mm, hl, lh; |m| <= 2^-8 |x|, |l| <= 2^-16 |x|).  The
// dropped ml + lm + ll is below 2^-23 |x y| and each part product is exact in
// FP32, so the result is as accurate as an FP32 product; the bf16 matrix rate
// is sixteen times the FP32 one.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// Split four FP32 values into their h, m and l parts, four bf16 each (8 bytes).
__device__ __forceinline__ void split3_bf16(const float (&x)[4], uint2& h, uint2& m, uint2& l) {
    uint32_t hw[2], mw[2], lw[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const f32x2_t v = {x[2 * p], x[2 * p + 1]};
        const bf16x2_t vh = __builtin_convertvector(v, bf16x2_t);
        const f32x2_t r1 = v - __builtin_convertvector(vh, f32x2_t);
        const bf16x2_t vm = __builtin_convertvector(r1, bf16x2_t);
        const f32x2_t r2 = r1 - __builtin_convertvector(vm, f32x2_t);
        const bf16x2_t vl = __builtin_convertvector(r2, bf16x2_t);
        hw[p] = __builtin_bit_cast(uint32_t, vh);
        mw[p] = __builtin_bit_cast(uint32_t, vm);
        lw[p] = __builtin_bit_cast(uint32_t, vl);
    }
    h = make_uint2(hw[0], hw[1]);
    m = make_uint2(mw[0], mw[1]);
    l = make_uint2(lw[0], lw[1]);
}

// One 16 x 16 x 32 step of a split product into c: the six part products of
// x = (h, m, l) and y, smallest first.  Lane layout as for the FP32 16x16x4
// instruction (row / column l % 16, result r of lane l at row 4 (l / 16) + r);
// lane group l / 16 supplies 8 k, the same k for x and y.
typedef float f32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f32x4_t mma_split6(const bf16x8_t (&x)[3], const bf16x8_t (&y)[3], f32x4_t c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[1], y[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[0], y[2], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[2], y[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[0], y[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[1], y[0], c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[0], y[0], c, 0, 0, 0);
}

// FP32 64 x 64 block products through the split bf16 form (above); off, they
// run on the FP32 matrix instructions.  (The split-K 32 x 32 kernel keeps the
// FP32 instructions: there the split's VALU work sits in each wave's serial
// path and measured slower at 512^2, 6.59 -> 7.09 us per product.)
constexpr bool kSplitBf16 = true;

// C = A Bt^T (MGemmArgs): a block owns a 32 x 32 tile of C and splits K over
// its kW waves (4 or 8); each wave accumulates the whole tile (2 x 2 MFMA
// 16x16 tiles) over its share of K, and the partial tiles are summed through
// LDS before the epilogue (by waves 0..3, one 16 x 16 quadrant each).  A and
// Bt are both k-contiguous.  Each wave stages its K range through its own LDS
// tile, one slice of 128 bytes per row at a time: 32 rows of A and of Bt copied with coalesced 16-byte loads (eight
// lanes per row, one cache line), the next slice's loads in flight while the
// current one is multiplied.  From LDS, lane group g = lane / 16 reads VEC
// consecutive k of its row per 16-byte read: k = STEP j + VEC g .. + VEC - 1
// (a permutation of K, the same for A and Bt), so one read feeds VEC
// instructions.
template <typename T>
struct NtCfg;
template <>
struct NtCfg<float> {
    static constexpr int VEC = 4;
};
template <>
struct NtCfg<double> {
    static constexpr int VEC = 2;
};
template <typename T, int kW = 4>
__device__ __forceinline__ void mgemm_body(const MGemmArgs<T>& a, int bx, int by, int gx) {
    using Cfg = MfmaCfg<T>;
    using acc_t = typename Cfg::acc_t;
    constexpr int VEC = NtCfg<T>::VEC, STEP = 4 * VEC;  // k consumed per round
    typedef T vec_t __attribute__((ext_vector_type(VEC)));
    __shared__ T red_tile[kW * 16 * 64];                // [wave][tile value][lane]
    __shared__ double red[17];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int M = a.M, N = a.N, K = a.K;
    // PCG state (done flag, stopping test): evaluated after the first operand
    // loads are in flight, so its latency overlaps theirs
    auto state_stops = [&]() -> bool {
        if (!a.st) return false;
        const int done = a.st->done;
        const double rrp = a.check ? partial_issue(a.rr_part, a.n_rr, tid, kW * 64) : 0.0;
        const double r0 = a.st->r0norm, tol = a.st->tol;
        const int cap = a.st->cap;
        if (done) return true;
        return a.check && pcg_stop_test(a.st, rrp, a.iter, r0, tol, cap, bx == 0 && by == 0 && tid == 0, red);
    };
    const int m0 = by * 32, n0 = bx * 32;
    const int g = lane >> 4, idx = lane & 15;
    using gvec_t = const gmem_t<vec_t>;
    const int kq = ((K + kW * STEP - 1) / (kW * STEP)) * STEP;  // this wave's share of K
    const int kbeg = wave * kq, kend = min(K, kbeg + kq);
    acc_t c00 = {}, c01 = {}, c10 = {}, c11 = {};
    // epilogue operands of this lane's four outputs, loaded with the first
    // operands rather than after the product (absent or outside C: ones for
    // E1, zeros for E2)
    const int ti = (wave & 3) >> 1, tj = wave & 1;
    const int jc = n0 + 16 * tj + idx;
    T e1v[4], e2v[4];
    {
        const bool has1 = a.epi >= 1 && a.E1, has2 = a.epi == 2;
        const gmem_t<T>* ones = gmem(nt_ones<T>());
        const gmem_t<T>* zeros = gmem(reinterpret_cast<const T*>(g_nt_zeros));
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = m0 + 16 * ti + Cfg::orow(lane, q);
            const bool in = i < M && jc < N;
            const size_t gidx = in ? size_t(i) * N + jc : 0;
            e1v[q] = *((in && has1) ? gmem(a.E1) + gidx : ones);
            e2v[q] = *((in && has2) ? gmem(a.E2) + gidx : zeros);
        }
    }
    {
        // per-wave LDS staging of this wave's K range: slices of BK k (128
        // bytes per row); the 16-byte chunk c of row r sits at c ^ ((r >> 1) & 7),
        // so the fragment reads of 16 consecutive rows and the row-chunk
        // stores both hit distinct banks
        constexpr int BK = 128 / int(sizeof(T)), LD = BK, CPR = BK / VEC;
        __shared__ __align__(16) T Ws[kW][2][32 * LD];
        T* As = Ws[wave][0];
        T* Bs = Ws[wave][1];
        const int rr = lane / CPR, cc = lane % CPR;  // rows rr + 8 h, chunk cc
        // rows outside the matrix feed only rows / columns of C that are not
        // stored: their addresses are clamped to row 0; k past the wave's
        // range loads as zero
        const gmem_t<T>* ra[4];
        const gmem_t<T>* rb[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int ia = m0 + rr + 8 * h, ib = n0 + rr + 8 * h;
            ra[h] = gmem(a.A) + size_t(ia < M ? ia : 0) * K;
            rb[h] = gmem(a.Bt) + size_t(ib < N ? ib : 0) * K;
        }
        vec_t la[4], lb[4];
        auto gload = [&](int k0) {
            const int k = k0 + cc * VEC;
            if (k0 + BK <= kend && (K % VEC) == 0) {
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    la[h] = *reinterpret_cast<gvec_t*>(ra[h] + k);
                    lb[h] = *reinterpret_cast<gvec_t*>(rb[h] + k);
                }
            } else {
#pragma unroll
                for (int h = 0; h < 4; ++h)
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const bool in = k + e < kend;
                        la[h][e] = in ? ra[h][k + e] : T(0);
                        lb[h][e] = in ? rb[h][k + e] : T(0);
                    }
            }
        };
        auto sstore = [&]() {
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int r = rr + 8 * h, sc = (cc ^ ((r >> 1) & 7)) * VEC;
                *reinterpret_cast<vec_t*>(As + r * LD + sc) = la[h];
                *reinterpret_cast<vec_t*>(Bs + r * LD + sc) = lb[h];
            }
        };
        const int sw = (idx >> 1) & 7;  // rows idx and idx + 16 share it
        const T* A0 = As + idx * LD;
        const T* B0 = Bs + idx * LD;
        auto compute = [&]() {
#pragma unroll
            for (int u = 0; u < BK / STEP; ++u) {
                const int c = ((g + 4 * u) ^ sw) * VEC;
                const vec_t fa0 = *reinterpret_cast<const vec_t*>(A0 + c);
                const vec_t fa1 = *reinterpret_cast<const vec_t*>(A0 + 16 * LD + c);
                const vec_t fb0 = *reinterpret_cast<const vec_t*>(B0 + c);
                const vec_t fb1 = *reinterpret_cast<const vec_t*>(B0 + 16 * LD + c);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    c00 = Cfg::mma(fa0[e], fb0[e], c00);
                    c01 = Cfg::mma(fa0[e], fb1[e], c01);
                    c10 = Cfg::mma(fa1[e], fb0[e], c10);
                    c11 = Cfg::mma(fa1[e], fb1[e], c11);
                }
            }
        };
        const int nsl = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
        if (nsl > 0) gload(kbeg);
        if (state_stops()) return;
        for (int sl = 0; sl < nsl; ++sl) {
            sstore();  // the wave's LDS reads of the previous slice are done (in-order LDS)
            if (sl + 1 < nsl) gload(kbeg + (sl + 1) * BK);
            compute();
        }
    }
    // sum the kW waves' partial tiles: wave w < 4 finishes tile (w / 2, w % 2)
    {
        T* mine = red_tile + wave * 16 * 64;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            mine[(0 * 4 + q) * 64 + lane] = c00[q];
            mine[(1 * 4 + q) * 64 + lane] = c01[q];
            mine[(2 * 4 + q) * 64 + lane] = c10[q];
            mine[(3 * 4 + q) * 64 + lane] = c11[q];
        }
    }
    __syncthreads();
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (wave >= 4) break;
        const int rv = (wave * 4 + q) * 64 + lane;
        T v0 = red_tile[rv] + red_tile[16 * 64 + rv];
        T v1 = red_tile[2 * 16 * 64 + rv] + red_tile[3 * 16 * 64 + rv];
        if constexpr (kW == 8) {
            v0 += red_tile[4 * 16 * 64 + rv] + red_tile[5 * 16 * 64 + rv];
            v1 += red_tile[6 * 16 * 64 + rv] + red_tile[7 * 16 * 64 + rv];
        }
        const T v = (v0 + v1) * e1v[q];  // e1v = 1 without a scale: exact
        const int i = m0 + 16 * ti + Cfg::orow(lane, q);
        if (i < M && jc < N) {
            const size_t gidx = size_t(i) * N + jc;
            if (a.transC) gmem(a.C)[size_t(jc) * M + i] = v;
            else gmem(a.C)[gidx] = v;
            if (a.epi == 2) part += double(e2v[q]) * double(v);
        }
    }
    if (a.epi == 2) {
        const double sm = block_sum(part, red);
        if (tid == 0) gmem(a.part)[by * gx + bx] = sm;
    }
}

// LDS layout of one operand tile of the split form (64 rows x 32 k, three bf16
// planes of 64 bytes per row) in 128-byte rows, as the FP32 tiles: row r of
// the first 8 KB holds plane h (chunks 0-3) and plane m (chunks 4-7) of tile
// row r; row r of the last 4 KB holds plane l of tile rows r and r + 32; the
// 16-byte chunk c of a 128-byte row q sits at c ^ ((q >> 1) & 7).
__device__ __forceinline__ int split_off(int plane, int r, int c) {
    const int q = plane < 2 ? r : (r & 31);
    const int chunk = plane < 2 ? 4 * plane + c : 4 * (r >> 5) + c;
    return (plane < 2 ? 0 : 64 * 128) + q * 128 + 16 * (chunk ^ ((q >> 1) & 7));
}

// 64 x 64 block tile staged through LDS: per K slice of 128 bytes per row
// (32 f32 / 16 f64), the block copies 64 rows of A and of Bt with coalesced
// 16-byte loads (eight lanes per row, one cache line) into a double-buffered
// LDS tile (16-byte chunks swizzled within each row, chunk c of row r at
// c ^ ((r >> 1) & 7): the fragment reads of 16 consecutive rows and the
// row-chunk stores hit distinct banks), and wave w multiplies its 32 x 32
// quadrant (w / 2, w % 2) from it: lane group g reads VEC consecutive k of its
// row per 16-byte read, one read feeding VEC instructions (the permutation of
// K of the direct kernel, shared by A and Bt).  One barrier per slice; the
// global loads of the next two slices are in flight while the current one is
// multiplied.
//
// Split form (FP32 with kSplitBf16): the copy stores each operand tile as three
// bf16 planes (h, m, l) of the slice's 32 k per row (split_off); lane group g
// reads chunk g (k = 8 g .. 8 g + 7) of its row of each plane, and one slice is
// one bf16 16x16x32 step: six instructions per 16 x 16 tile.
//
// kG = 2: eight waves in two K groups, each with its own LDS buffers; group
// g takes slices g, g + 2, ... (both groups run the same number of steps, the
// second one's last slice past K reading zeros), and group 1 adds its tile
// to group 0's through LDS before the epilogue.  Twice the waves per CU for
// grids of about one block per CU.
template <typename T, int kG = 1>
__device__ __forceinline__ void mgemm_lds_body(const MGemmArgs<T>& a, int bx, int by, int gx) {
    using Cfg = MfmaCfg<T>;
    using acc_t = typename Cfg::acc_t;
    constexpr bool SPLIT = kSplitBf16 && std::is_same<T, float>::value;
    constexpr int VEC = NtCfg<T>::VEC, STEP = 4 * VEC;
    constexpr int BK = 128 / int(sizeof(T));      // k per slice
    constexpr int LD = BK;                        // row (elements); 16-byte chunks swizzled
    constexpr int CPR = BK / VEC;                 // 16-byte chunks per row (8)
    typedef T vec_t __attribute__((ext_vector_type(VEC)));
    // per operand and buffer: the T tile (64 rows x 128 bytes), or three bf16
    // planes of 64 rows x 64 bytes
    constexpr int TILE_BYTES = SPLIT ? 3 * 64 * 64 : 64 * LD * int(sizeof(T));
    __shared__ __align__(16) unsigned char smem_all[kG * 4 * TILE_BYTES];
    __shared__ double red[17];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = wave >> 2, gtid = tid & 255;  // K group, thread in the group
    unsigned char* const smem = smem_all + grp * 4 * TILE_BYTES;
    T (*As)[64 * LD] = reinterpret_cast<T (*)[64 * LD]>(smem);
    T (*Bs)[64 * LD] = reinterpret_cast<T (*)[64 * LD]>(smem + 2 * TILE_BYTES);
    const int M = a.M, N = a.N, K = a.K;
    const int bm = by * 64, bn = bx * 64;
    // this thread's two 16-byte chunks of each operand tile (h = 0, 1): rows
    // r0 and r0 + 32 at chunk cc; in the split form one row, rs, and the two
    // chunks of its 8 k from 8 c8 (one 16-byte store per bf16 plane)
    const int r0 = gtid / CPR, cc = gtid % CPR;
    const int rs = gtid >> 2, c8 = gtid & 3;
    int kk[2];  // the chunks' k within a slice
    const gmem_t<T>* pa[2];
    const gmem_t<T>* pb[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int rr = SPLIT ? rs : r0 + 32 * h;
        kk[h] = SPLIT ? 8 * c8 + 4 * h : cc * VEC;
        const int ra = bm + rr, rb = bn + rr;
        pa[h] = gmem(a.A) + size_t(ra < M ? ra : 0) * K;
        pb[h] = gmem(a.Bt) + size_t(rb < N ? rb : 0) * K;
    }
    vec_t va[2][2], vb[2][2];  // [register slot][chunk h]
    // Rows of whole 16-byte chunks (K % VEC == 0): one 16-byte load per chunk
    // and operand for every slice, chunks past K read from a 16-byte block of
    // zeros (an address select: no branch and no select on a loaded value, so
    // the wait before a copy covers only the loads that copy needs).
    const gmem_t<vec_t>* zchunk = reinterpret_cast<const gmem_t<vec_t>*>(gmem(g_nt_zeros));
    auto gload_al = [&](int k0, int slot) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = k0 + kk[h];
            const bool in = k < K;
            va[slot][h] = *(in ? reinterpret_cast<const gmem_t<vec_t>*>(pa[h] + k) : zchunk);
            vb[slot][h] = *(in ? reinterpret_cast<const gmem_t<vec_t>*>(pb[h] + k) : zchunk);
        }
        // keep the loads here: moved up by the compiler, they shared
        // registers with the fragment reads and every slice waited for them
        asm volatile("" ::: "memory");
    };
    // Other K: element loads past the last whole slice, zeros past K.
    auto gload = [&](int k0, int slot) {
        if (k0 + BK <= K && (K % VEC) == 0) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                va[slot][h] = *reinterpret_cast<const gmem_t<vec_t>*>(pa[h] + k0 + kk[h]);
                vb[slot][h] = *reinterpret_cast<const gmem_t<vec_t>*>(pb[h] + k0 + kk[h]);
            }
        } else {  // tail slice: zeros past K
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int k = k0 + kk[h] + e;
                    const bool in = k < K;
                    va[slot][h][e] = in ? pa[h][k] : T(0);
                    vb[slot][h][e] = in ? pb[h][k] : T(0);
                }
        }
    };
    auto sstore = [&](int buf, int slot) {
        // the split of a slot stays after the copy before it: scheduled
        // earlier, it waited for loads issued half a step before
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (SPLIT) {
            // 8 k of row rs: chunk c8 of each plane, one 16-byte store each
            auto put3 = [&](const vec_t (&x)[2], unsigned char* t) {
                uint2 h0, m0, l0, h1, m1, l1;
                const float x0[4] = {x[0][0], x[0][1], x[0][2], x[0][3]};
                const float x1[4] = {x[1][0], x[1][1], x[1][2], x[1][3]};
                split3_bf16(x0, h0, m0, l0);
                split3_bf16(x1, h1, m1, l1);
                *reinterpret_cast<uint4*>(t + split_off(0, rs, c8)) = make_uint4(h0.x, h0.y, h1.x, h1.y);
                *reinterpret_cast<uint4*>(t + split_off(1, rs, c8)) = make_uint4(m0.x, m0.y, m1.x, m1.y);
                *reinterpret_cast<uint4*>(t + split_off(2, rs, c8)) = make_uint4(l0.x, l0.y, l1.x, l1.y);
            };
            put3(va[slot], smem + buf * TILE_BYTES);
            put3(vb[slot], smem + (2 + buf) * TILE_BYTES);
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int r = r0 + 32 * h, sc = (cc ^ ((r >> 1) & 7)) * VEC;
                *reinterpret_cast<vec_t*>(&As[buf][r * LD + sc]) = va[slot][h];
                *reinterpret_cast<vec_t*>(&Bs[buf][r * LD + sc]) = vb[slot][h];
            }
        }
    };
    const int g = lane >> 4, idx = lane & 15;
    const int wm = ((wave & 3) >> 1) * 32, wn = (wave & 1) * 32;
    acc_t c00 = {}, c01 = {}, c10 = {}, c11 = {};
    auto compute_split = [&](int buf) {
        if constexpr (SPLIT) {
            // rows wm + idx and wm + idx + 16 of A, wn + idx (+16) of Bt
            const unsigned char* ta = smem + buf * TILE_BYTES;
            const unsigned char* tb = smem + (2 + buf) * TILE_BYTES;
            bf16x8_t fa[2][3], fb[2][3];  // [row half][plane h, m, l]
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    fa[hh][q] = *reinterpret_cast<const bf16x8_t*>(ta + split_off(q, wm + idx + 16 * hh, g));
                    fb[hh][q] = *reinterpret_cast<const bf16x8_t*>(tb + split_off(q, wn + idx + 16 * hh, g));
                }
            c00 = mma_split6(fa[0], fb[0], c00);
            c01 = mma_split6(fa[0], fb[1], c01);
            c10 = mma_split6(fa[1], fb[0], c10);
            c11 = mma_split6(fa[1], fb[1], c11);
        }
    };
    auto compute = [&](int buf) {
        if constexpr (SPLIT) {
            compute_split(buf);
            return;
        }
        // rows wm + idx (+16): (row >> 1) & 7 is the same for row and row + 16
        const int sa = ((wm + idx) >> 1) & 7, sb = ((wn + idx) >> 1) & 7;
        const T* A0 = &As[buf][(wm + idx) * LD];
        const T* A1 = A0 + 16 * LD;
        const T* B0 = &Bs[buf][(wn + idx) * LD];
        const T* B1 = B0 + 16 * LD;
#pragma unroll
        for (int u = 0; u < BK / STEP; ++u) {
            const int ca = ((g + 4 * u) ^ sa) * VEC, cb = ((g + 4 * u) ^ sb) * VEC;
            const vec_t fa0 = *reinterpret_cast<const vec_t*>(A0 + ca);
            const vec_t fa1 = *reinterpret_cast<const vec_t*>(A1 + ca);
            const vec_t fb0 = *reinterpret_cast<const vec_t*>(B0 + cb);
            const vec_t fb1 = *reinterpret_cast<const vec_t*>(B1 + cb);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                c00 = Cfg::mma(fa0[e], fb0[e], c00);
                c01 = Cfg::mma(fa0[e], fb1[e], c01);
                c10 = Cfg::mma(fa1[e], fb0[e], c10);
                c11 = Cfg::mma(fa1[e], fb1[e], c11);
            }
        }
    };
    // PCG state: evaluated while the first slices are in flight
    auto state_stops = [&]() -> bool {
        if (!a.st) return false;
        const int done = a.st->done;
        const double rrp = a.check ? partial_issue(a.rr_part, a.n_rr, tid, 256 * kG) : 0.0;
        const double r0n = a.st->r0norm, tol = a.st->tol;
        const int cap = a.st->cap;
        if (done) return true;
        return a.check && pcg_stop_test(a.st, rrp, a.iter, r0n, tol, cap, bx == 0 && by == 0 && tid == 0, red);
    };
    const int nsl = (K + BK - 1) / BK;
    const int J = (nsl + kG - 1) / kG;  // steps (slices per group)
    // k of the group's j-th slice (the last one again past its last step)
    auto kof = [&](int j) { return (grp + kG * min(j, J - 1)) * BK; };
    if ((K % VEC) == 0) {
        // slice j is loaded into register slot j & 1 two slices ahead of its
        // use and copied to LDS buffer j & 1 one slice ahead; the loop is
        // unrolled by two so that the slots are static, and its body has no
        // conditional step (past the last slice the loads repeat it, unused)
        gload_al(kof(0), 0);
        gload_al(kof(1), 1);
        if (state_stops()) return;
        sstore(0, 0);
        __syncthreads();
        gload_al(kof(2), 0);
        int j = 0;
        for (; j + 2 < J; j += 2) {  // LDS buffer 0: step j
            compute(0);
            sstore(1, 1);  // step j + 1
            __syncthreads();
            gload_al(kof(j + 3), 1);
            compute(1);
            sstore(0, 0);  // step j + 2
            __syncthreads();
            gload_al(kof(j + 4), 0);
        }
        compute(0);  // step j, then step j + 1 if there is one
        if (j + 1 < J) {
            sstore(1, 1);
            __syncthreads();
            compute(1);
        }
    } else {
        // one slice ahead, in register slot 0
        gload(kof(0), 0);
        if (state_stops()) return;
        sstore(0, 0);
        __syncthreads();
        for (int j = 0; j < J; ++j) {
            if (j + 1 < J) gload(kof(j + 1), 0);
            compute(j & 1);
            if (j + 1 < J) sstore((j + 1) & 1, 0);
            __syncthreads();
        }
    }
    if constexpr (kG == 2) {
        // group 1's tile into group 0's accumulators (through the group LDS
        // buffers, free once every wave has passed the barrier below)
        __syncthreads();
        T* racc = reinterpret_cast<T*>(smem_all) + (wave & 3) * 16 * 64 + lane;
        if (grp == 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                racc[(0 * 4 + q) * 64] = c00[q];
                racc[(1 * 4 + q) * 64] = c01[q];
                racc[(2 * 4 + q) * 64] = c10[q];
                racc[(3 * 4 + q) * 64] = c11[q];
            }
        }
        __syncthreads();
        if (grp == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                c00[q] += racc[(0 * 4 + q) * 64];
                c01[q] += racc[(1 * 4 + q) * 64];
                c10[q] += racc[(2 * 4 + q) * 64];
                c11[q] += racc[(3 * 4 + q) * 64];
            }
        }
    }
    // epilogue: each wave stores its quadrant
    const int m0 = bm + wm, n0 = bn + wn;
    const bool has1 = a.epi >= 1 && a.E1;
    double part = 0.0;
    auto put = [&](const acc_t& c, int ri, int cj) {
        const int j = n0 + 16 * cj + idx;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = m0 + 16 * ri + Cfg::orow(lane, q);
            if (i < M && j < N) {
                const size_t gidx = size_t(i) * N + j;
                const T v = has1 ? c[q] * gmem(a.E1)[gidx] : c[q];
                if (a.transC) gmem(a.C)[size_t(j) * M + i] = v;
                else gmem(a.C)[gidx] = v;
                if (a.epi == 2) part += double(gmem(a.E2)[gidx]) * double(v);
            }
        }
    };
    if (grp == 0) {
        put(c00, 0, 0);
        put(c01, 0, 1);
        put(c10, 1, 0);
        put(c11, 1, 1);
    }
    if (a.epi == 2) {
        const double sm = block_sum(part, red);
        if (tid == 0) gmem(a.part)[by * gx + bx] = sm;
    }
}

// Waves per block of the single-image split-K product: 8 for FP64 (half the
// FP32 matrix rate and half the k per 16-byte LDS read, so a second wave per
// SIMD overlaps one wave's reads with the other's MFMAs: 8% off the FP64
// restore at 512^2), 4 for FP32 (8 measured no faster).
template <typename T>
constexpr int kMgemmWaves = sizeof(T) == 8 ? 8 : 4;

template <typename T>
__global__ void __launch_bounds__(512) k_mgemm(MGemmArgs<T> a) {
    int bx, by;
    tile_of_block(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x, gridDim.y, bx, by);
    mgemm_body<T, kMgemmWaves<T>>(a, bx, by, gridDim.x);
}

// Single-image 64 x 64 products: two K groups (about one block per CU at the
// sizes where this tile is chosen).
template <typename T>
__global__ void __launch_bounds__(512) k_mgemm64(MGemmArgs<T> a) {
    int bx, by;
    tile_of_block(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x, gridDim.y, bx, by);
    mgemm_lds_body<T, 2>(a, bx, by, gridDim.x);
}

// Batched products: image blockIdx.z, its own tile grid inside the launch
// grid; images whose PCG has stopped skip their blocks.  it: PCG iteration.
// One kernel per block tile (each with only its own LDS).
template <typename T, int kTile>
__global__ void __launch_bounds__(256) k_mgemm_b(const MGemmArgs<T>* __restrict__ as, int it) {
    MGemmArgs<T> a = as[blockIdx.z];
    const int gx = (a.N + kTile - 1) / kTile, gy = (a.M + kTile - 1) / kTile;
    const int b = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int bx = b % gridDim.x, by = b / gridDim.x;
    if (bx >= gx || by >= gy || (a.st && a.st->done)) return;
    a.iter = it;
    if constexpr (kTile == 64) mgemm_lds_body<T>(a, bx, by, gx);
    else mgemm_body<T>(a, bx, by, gx);
}

template <typename T, int kTile>
__global__ void __launch_bounds__(256) k_mgemm_bc(const MGemmArgs<T>* __restrict__ as, int it,
                                                  const int* __restrict__ prefix, int count) {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int img = batch_image(prefix, count, b);
    MGemmArgs<T> a = as[img];
    if (a.st && a.st->done) return;
    a.iter = it;
    const int gx = (a.N + kTile - 1) / kTile;
    const int local = b - prefix[img];
    if constexpr (kTile == 64) mgemm_lds_body<T>(a, local % gx, local / gx, gx);
    else mgemm_body<T>(a, local % gx, local / gx, gx);
}

// FP64 sums of products C = sum_t coef_t op(A_t) B_t on the matrix cores
// (the eigenvalue setup); one problem per blockIdx.z, 32 x 32 tiles.  With
// transA, A_t is stored K x M and its slice is loaded along m.
__global__ void __launch_bounds__(256) k_mgemm_multi(const GemmProblem* __restrict__ probs) {
    using Cfg = MfmaCfg<double>;
    constexpr int BK = Cfg::BK, SA = Cfg::SA, SB = Cfg::SB, TM = 32, TN = 32;
    constexpr int AE = TM * BK / 256, BE = BK * TN / 256;
    __shared__ double As[2][TM * SA];
    __shared__ double Bs[2][BK * SB];
    const GemmProblem& pb = probs[blockIdx.z];
    const int M = pb.M, N = pb.N, K = pb.K;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    if (m0 >= M || n0 >= N) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int trans = pb.transA;
    // A slice: row-major -> thread (row ar, k ak..); stored K x M -> thread (k kk, rows rr..)
    const int ar = tid / (BK / AE), ak = (tid % (BK / AE)) * AE;
    const int kk = tid / (TM / AE), rr = (tid % (TM / AE)) * AE;
    const int bk = tid / (TN / BE), bc = (tid % (TN / BE)) * BE;
    const int nkt = (K + BK - 1) / BK, total = pb.nterms * nkt;
    double ra[AE], rb[BE];
    // whole tiles and whole K slices (uniform): the loads need no masks
    const bool whole = m0 + TM <= M && n0 + TN <= N && K % BK == 0;
    auto gload_whole = [&](int step) {
        const int term = step / nkt, k0 = (step - term * nkt) * BK;
        const double* A = pb.t[term].A;
        const double* B = pb.t[term].B;
        const double cf = pb.t[term].coef;
        if (trans) {
#pragma unroll
            for (int c = 0; c < AE; ++c) ra[c] = cf * A[size_t(k0 + kk) * M + m0 + rr + c];
        } else {
#pragma unroll
            for (int c = 0; c < AE; ++c) ra[c] = cf * A[size_t(m0 + ar) * K + k0 + ak + c];
        }
#pragma unroll
        for (int c = 0; c < BE; ++c) rb[c] = B[size_t(k0 + bk) * N + n0 + bc + c];
    };
    auto gload_masked = [&](int step) {
        const int term = step / nkt, k0 = (step - term * nkt) * BK;
        const double* A = pb.t[term].A;
        const double* B = pb.t[term].B;
        const double cf = pb.t[term].coef;
        if (trans) {
            const int gk = k0 + kk;
#pragma unroll
            for (int c = 0; c < AE; ++c) {
                const int gm = m0 + rr + c;
                ra[c] = (gk < K && gm < M) ? cf * A[size_t(gk) * M + gm] : 0.0;
            }
        } else {
            const int gr = m0 + ar;
#pragma unroll
            for (int c = 0; c < AE; ++c) {
                const int gk = k0 + ak + c;
                ra[c] = (gr < M && gk < K) ? cf * A[size_t(gr) * K + gk] : 0.0;
            }
        }
        const int gk = k0 + bk;
#pragma unroll
        for (int c = 0; c < BE; ++c) {
            const int gc = n0 + bc + c;
            rb[c] = (gk < K && gc < N) ? B[size_t(gk) * N + gc] : 0.0;
        }
    };
    auto gload = [&](int step) {
        if (whole) gload_whole(step);
        else gload_masked(step);
    };
    auto sstore = [&](int buf) {
        if (trans) {
#pragma unroll
            for (int c = 0; c < AE; ++c) As[buf][(rr + c) * SA + kk] = ra[c];
        } else {
#pragma unroll
            for (int c = 0; c < AE; ++c) As[buf][ar * SA + ak + c] = ra[c];
        }
#pragma unroll
        for (int c = 0; c < BE; ++c) Bs[buf][bk * SB + bc + c] = rb[c];
    };
    Cfg::acc_t acc = {};
    const int wr = (wave >> 1) * 16, wc = (wave & 1) * 16;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int step = 0; step < total; ++step) {
        const int buf = step & 1;
        if (step + 1 < total) gload(step + 1);
        mma_slice<double>(As[buf], Bs[buf], lane, wr, wc, acc);
        if (step + 1 < total) sstore(buf ^ 1);
        __syncthreads();
    }
    const int j = n0 + wc + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = m0 + wr + Cfg::orow(lane, r);
        if (i < M && j < N) pb.C[size_t(i) * N + j] = acc[r];
    }
}

// x += a p, r -= a q, ||r||^2 partials, t = s o r (see UpdArgs).  Each
// thread owns kUpdE elements (stride 256 inside the block's range); all its
// loads are issued before the scalar reductions.
constexpr int kUpdE = 4;
template <typename T>
__device__ __forceinline__ void upd_body(const UpdArgs<T>& a, int bx) {
    __shared__ double red[17];
    const int tid = threadIdx.x;
    const int base = bx * 256 * kUpdE + tid;
    const int done = a.st->done;
    const double pq = a.do_update ? partial_issue(a.pq_part, a.n_pq, tid, 256) : 0.0;
    const double rzp = a.do_update ? partial_issue(a.rz_part, a.n_rz, tid, 256) : 0.0;
    T rv[kUpdE], qv[kUpdE], xv[kUpdE], pv[kUpdE], sv[kUpdE];
#pragma unroll
    for (int c = 0; c < kUpdE; ++c) {
        const int k = base + 256 * c;
        const bool in = k < a.n;
        rv[c] = in ? a.r[k] : T(0);
        sv[c] = (in && a.s) ? a.s[k] : T(1);
        if (a.do_update) {
            qv[c] = in ? a.q[k] : T(0);
            xv[c] = in ? a.x[k] : T(0);
            pv[c] = in ? a.p[k] : T(0);
        }
    }
    if (done) return;
    T step = T(0);
    if (a.do_update) {
        const double g = block_sum(pq, red);
        const double rz = block_sum(rzp, red);
        if (!(g > 0.0)) {  // curvature <= 0 (or NaN): stop, keep x_{i-1}
            if (bx == 0 && tid == 0) {
                a.st->done = 2;
                a.st->iters = a.iter - 1;
            }
            return;
        }
        step = T(rz / g);
    }
    double part = 0.0;
#pragma unroll
    for (int c = 0; c < kUpdE; ++c) {
        const int k = base + 256 * c;
        if (k >= a.n) continue;
        T r = rv[c];
        if (a.do_update) {
            r -= step * qv[c];
            a.x[k] = xv[c] + step * pv[c];
            a.r[k] = r;
            part += double(r) * double(r);
        }
        a.t[k] = sv[c] * r;
    }
    if (a.do_update) {
        const double sm = block_sum(part, red);
        if (tid == 0) a.rr_out[bx] = sm;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_upd(UpdArgs<T> a) {
    upd_body(a, blockIdx.x);
}

__host__ __device__ constexpr int upd_blocks(int n) {
    return (n + 256 * kUpdE - 1) / (256 * kUpdE);
}

template <typename T>
__global__ void __launch_bounds__(256) k_upd_b(const UpdArgs<T>* __restrict__ as, int it) {
    UpdArgs<T> a = as[blockIdx.z];
    if (int(blockIdx.x) >= upd_blocks(a.n) || a.st->done) return;
    a.iter = it;
    upd_body(a, blockIdx.x);
}

// w = (I (x) K_x) z, one row per block; the z row and the band's rows
// (interior Toeplitz row, then the stored edge rows) are staged in LDS.
template <typename T>
__device__ __forceinline__ void xpass_body(const XPassArgs<T>& a, int i) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* zs = reinterpret_cast<T*>(smem_raw);
    const int nx = a.nx;
    T* cs = zs + nx;
    const int tid = threadIdx.x;
    const T* zr = a.z + size_t(i) * nx;
    for (int t = tid; t < nx; t += 256) zs[t] = zr[t];
    for (int t = tid; t < a.xband_len; t += 256) cs[t] = a.xband[t];
    if (a.st && a.st->done) return;  // after the loads: their latencies overlap
    __syncthreads();
    const int bw = 2 * a.kw + 1;
    for (int t = tid; t < nx; t += 256) {
        const int rr = t < a.klo ? 1 + t : (t >= a.khi ? 1 + a.klo + (t - a.khi) : 0);
        const T* coef = cs + rr * bw;
        T sacc = T(0);
        for (int d = 0; d < bw; ++d) sacc += coef[d] * zs[min(max(t + d - a.kw, 0), nx - 1)];
        a.w[size_t(i) * nx + t] = sacc;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_xpass(XPassArgs<T> a) {
    xpass_body(a, blockIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(256) k_xpass_b(const XPassArgs<T>* __restrict__ as) {
    const XPassArgs<T> a = as[blockIdx.z];
    if (int(blockIdx.x) >= a.ny) return;
    xpass_body(a, blockIdx.x);
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
__device__ __forceinline__ void kappa_at(int i, int j, int ny, int nx, const T* __restrict__ u, double alpha,
                                         double beta, int variant, T* kap, double* kapd, T* s_apply, double* s_mu,
                                         double* Dd) {
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

template <typename T>
__global__ void k_kappa(int ny, int nx, const T* __restrict__ u, double alpha, double beta, int variant,
                        T* kap, double* kapd, T* s_apply, double* s_mu, double* Dd) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= nx) return;
    kappa_at(i, j, ny, nx, u, alpha, beta, variant, kap, kapd, s_apply, s_mu, Dd);
}

template <typename T>
__global__ void k_kappa_b(const KappaArgs<T>* __restrict__ as) {
    const KappaArgs<T> a = as[blockIdx.z];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (i >= a.ny || j >= a.nx) return;
    kappa_at(i, j, a.ny, a.nx, a.u, a.alpha, a.beta, a.variant, a.kap, a.kapd, a.s_apply, a.s_mu, a.Dd);
}

// L(u^k) under anti-reflective BCs (the reblurring system's AR L): the
// diffusivity on every face of the image, the ghost faces included, from the
// anti-reflectively extended u^k (one ghost line per side, rows first, then
// columns; on a row face the y-difference of the cell above it, on a column
// face the x-difference of the cell left of it), folded into the four
// coefficients of a 5-point stencil per pixel:
//   (L y)_ij = cu (y_ij - y_i-1,j) + cd (y_ij - y_i+1,j) + cl (y_ij - y_i,j-1) + cr (y_ij - y_i,j+1)
// interior rows: cu = kx(face above), cd = kx(face below); row 0: cu = 0,
// cd = kx(face 1) - kx(ghost face 0) (the ghost flux reflects the first
// difference); the last row: cu = kx(its upper face) - kx(ghost face),
// cd = 0; columns alike.  Needs ny, nx >= 3.
template <typename T>
__global__ void k_kappa_ar(int ny, int nx, const T* __restrict__ u, double beta, double* cu, double* cd,
                           double* cl, double* cr, T* cut, T* cdt, T* clt, T* crt) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= nx) return;
    const double b2 = beta * beta;
    auto R = [&](int r, int c) -> double {  // rows extended, c in [0, nx)
        if (r < 0) return 2.0 * double(u[c]) - double(u[size_t(nx) + c]);
        if (r >= ny) return 2.0 * double(u[size_t(ny - 1) * nx + c]) - double(u[size_t(ny - 2) * nx + c]);
        return double(u[size_t(r) * nx + c]);
    };
    auto E = [&](int r, int c) -> double {  // then columns
        if (c < 0) return 2.0 * R(r, 0) - R(r, 1);
        if (c >= nx) return 2.0 * R(r, nx - 1) - R(r, nx - 2);
        return R(r, c);
    };
    // face f between rows f-1 and f (f = 0..ny), column j
    auto KX = [&](int f) {
        const double gx = E(f, j) - E(f - 1, j), gy = E(f - 1, j + 1) - E(f - 1, j);
        return 1.0 / sqrt(gx * gx + gy * gy + b2);
    };
    // face f between columns f-1 and f (f = 0..nx), row i
    auto KY = [&](int f) {
        const double gy = E(i, f) - E(i, f - 1), gx = E(i + 1, f - 1) - E(i, f - 1);
        return 1.0 / sqrt(gx * gx + gy * gy + b2);
    };
    double vu, vd, vl, vr;
    if (i == 0) {
        vu = 0.0;
        vd = KX(1) - KX(0);
    } else if (i == ny - 1) {
        vu = KX(ny - 1) - KX(ny);
        vd = 0.0;
    } else {
        vu = KX(i);
        vd = KX(i + 1);
    }
    if (j == 0) {
        vl = 0.0;
        vr = KY(1) - KY(0);
    } else if (j == nx - 1) {
        vl = KY(nx - 1) - KY(nx);
        vr = 0.0;
    } else {
        vl = KY(j);
        vr = KY(j + 1);
    }
    const size_t g = size_t(i) * nx + j;
    cu[g] = vu;
    cd[g] = vd;
    cl[g] = vl;
    cr[g] = vr;
    cut[g] = T(vu);
    cdt[g] = T(vd);
    clt[g] = T(vl);
    crt[g] = T(vr);
}

__device__ __forceinline__ void operands_at(int i, int j, int ny, int nx, const double* __restrict__ kap,
                                            const double* __restrict__ s, double* A1, double* A2, double* A3,
                                            double* B1, double* B2, double* B3) {
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

__global__ void k_gemm_operands(int ny, int nx, const double* __restrict__ kap, const double* __restrict__ s,
                                double* A1, double* A2, double* A3, double* B1, double* B2, double* B3) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= nx) return;
    operands_at(i, j, ny, nx, kap, s, A1, A2, A3, B1, B2, B3);
}

__global__ void k_operands_b(const OperandArgs* __restrict__ as) {
    const OperandArgs a = as[blockIdx.z];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (i >= a.ny || j >= a.nx) return;
    operands_at(i, j, a.ny, a.nx, a.kapd, a.s_mu, a.A1, a.A2, a.A3, a.B1, a.B2, a.B3);
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
__global__ void k_mu_b(const MuArgs<T>* __restrict__ as) {
    const MuArgs<T> a = as[blockIdx.z];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    double h2 = a.lamh2[k];
    if (a.use_lamd) h2 *= a.lamd[k] * a.lamd[k];
    const double m = h2 + a.alpha * (a.lamx[k] + a.lamy[k]);
    a.mu[k] = m;
    a.muinv[k] = T(1.0 / m);
}

template <typename T>
__global__ void k_fpchange_b(const FpArgs<T>* __restrict__ as) {
    __shared__ double red[17];
    const FpArgs<T> a = as[blockIdx.z];
    if (int(blockIdx.x) >= a.nb) return;
    double s1 = 0.0, s2 = 0.0;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < a.n; k += a.nb * blockDim.x) {
        const double xv = a.x[k], d = xv - double(a.u[k]);
        s1 += d * d;
        s2 += xv * xv;
    }
    const double t1 = block_sum(s1, red);
    const double t2 = block_sum(s2, red);
    if (threadIdx.x == 0) {
        a.part[2 * blockIdx.x] = t1;
        a.part[2 * blockIdx.x + 1] = t2;
    }
}

template <typename T>
__global__ void k_copy_b(const CopyArgs<T>* __restrict__ as) {
    const CopyArgs<T> a = as[blockIdx.z];
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < a.n; k += gridDim.x * blockDim.x) a.dst[k] = a.src[k];
}

// Per-block FP64 partials of the TV objective of eq. (mp),
// T(u) = 1/2 ||H u - v||^2 + alpha sum sqrt(|D u|^2 + beta^2), from H u (FP64).
template <typename T>
__global__ void k_objective(int ny, int nx, const double* __restrict__ hu, const T* __restrict__ v,
                            const T* __restrict__ u, double alpha, double beta, double* part) {
    __shared__ double red[17];
    const size_t n = size_t(ny) * nx;
    double acc = 0.0;
    for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < n; g += size_t(gridDim.x) * blockDim.x) {
        const int i = int(g / nx), j = int(g - size_t(i) * nx);
        const double c = u[g], r = hu[g] - double(v[g]);
        const double dx = i < ny - 1 ? double(u[g + nx]) - c : 0.0;
        const double dy = j < nx - 1 ? double(u[g + 1]) - c : 0.0;
        acc += 0.5 * r * r + alpha * sqrt(dx * dx + dy * dy + beta * beta);
    }
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
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

__device__ __forceinline__ void finalize_body(PcgState* st, const double* rr_part, int n_rr, const double* fp_part,
                                              int n_fp, int max_iter) {
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

__global__ void k_finalize_b(const FinArgs* __restrict__ as) {
    const FinArgs a = as[blockIdx.x];
    finalize_body(a.st, a.rr_part, a.n_rr, a.fp_part, a.n_fp, a.max_iter);
}

__global__ void k_init_b(const InitArgs* __restrict__ as) {
    const InitArgs a = as[blockIdx.x];
    if (threadIdx.x != 0) return;
    a.st->r0norm = 0.0;
    a.st->tol = a.tol;
    a.st->relres = 0.0;
    a.st->fp_change = 0.0;
    a.st->done = a.frozen ? 3 : 0;
    a.st->iters = 0;
    a.st->cap = a.cap;
}

__global__ void k_init_state(PcgState* st, double tol) {
    st->r0norm = 0.0;
    st->tol = tol;
    st->relres = 0.0;
    st->fp_change = 0.0;
    st->done = 0;
    st->iters = 0;
    st->cap = 0;
}

// Adjoint step: vbar += H lambda; e = D_x lam o D_x u^{k+1} + D_y lam o
// D_y u^{k+1}; g = kappa^3 e; partials of sum kappa e and sum kappa^3 e.
template <typename T>
__global__ void k_adj_accum(int ny, int nx, const T* __restrict__ lam, const T* __restrict__ hlam,
                            const T* __restrict__ u1, const double* __restrict__ kap, double* vbar, double* g,
                            double* part) {
    __shared__ double red[17];
    double s1 = 0.0, s3 = 0.0;
    const int n = ny * nx;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const int i = k / nx, j = k - i * nx;
        const double lc = lam[k], uc = u1[k];
        double e = 0.0;
        if (i < ny - 1) e += (double(lam[k + nx]) - lc) * (double(u1[k + nx]) - uc);
        if (j < nx - 1) e += (double(lam[k + 1]) - lc) * (double(u1[k + 1]) - uc);
        const double kc = kap[k];
        const double k3e = kc * kc * kc * e;
        s1 += kc * e;
        s3 += k3e;
        g[k] = k3e;
        vbar[k] += double(hlam[k]);
    }
    const double a = block_sum(s1, red);
    const double b = block_sum(s3, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// ubar^k = alpha [D_x^T (g o D_x u^k) + D_y^T (g o D_y u^k)].
template <typename T>
__global__ void k_adj_ubar(int ny, int nx, const double* __restrict__ g, const T* __restrict__ u, double alpha,
                           double* ubar) {
    const int n = ny * nx;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const int i = k / nx, j = k - i * nx;
        const double uc = u[k];
        double s = 0.0;
        if (i > 0) s += g[k - nx] * (uc - double(u[k - nx]));
        if (i < ny - 1) s -= g[k] * (double(u[k + nx]) - uc);
        if (j > 0) s += g[k - 1] * (uc - double(u[k - 1]));
        if (j < nx - 1) s -= g[k] * (double(u[k + 1]) - uc);
        ubar[k] = alpha * s;
    }
}

template <typename T>
__global__ void k_cast_from_double(int n, const double* src, T* dst) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = T(src[k]);
}

template <typename T>
__global__ void k_add_to_double(int n, const T* src, double* dst) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] += double(src[k]);
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
    tvd_launch((k_band<TX, TS, T, TY>), grid, dim3(kBandThreads), lds, s, a);
    return hipGetLastError();
}

template <typename T>
LineGeom line_geom(int lines, int n, int M) {
    LineGeom g;
    g.units = (lines + 1) / 2;
    // one radix-8 butterfly per thread per stage, and each thread holds at
    // most kLinePos positions of a line of length n
    // (one position per thread where possible: shorter serial load/store phases)
    g.tpu = std::min(256, std::max(64, M / 8));
    while (g.tpu < n && g.tpu < 1024) g.tpu *= 2;
    if (g.tpu * kLinePos < n) g.tpu = 0;  // line too long for one block
    const size_t per_unit = size_t(2) * padded_len(M) * sizeof(cx<T>);
    int upb = std::max(1, 256 / g.tpu);
    while (upb > 1 && per_unit * upb > 80 * 1024) upb >>= 1;
    g.upb = std::min(upb, g.units);
    g.blocks = (g.units + g.upb - 1) / g.upb;
    g.lds = per_unit * g.upb;
    return g;
}

template <typename T>
size_t lds_table_bytes(int blob_len) {
    return size_t(lds_table_len<T>(blob_len)) * sizeof(cx<T>);
}

template <typename T>
hipError_t launch_rowpass(const RowPassArgs<T>& a, hipStream_t s) {
    auto k = a.plan.tables_in_lds ? &k_rowpass<T, true> : &k_rowpass<T, false>;
    if (a.g.lds > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  int(a.g.lds));
    tvd_launch(k, dim3(a.g.blocks), dim3(a.g.upb * a.g.tpu), a.g.lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_colpass(const ColPassArgs<T>& a, hipStream_t s) {
    auto k = a.plan.tables_in_lds ? &k_colpass<T, true> : &k_colpass<T, false>;
    if (a.g.lds > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  int(a.g.lds));
    tvd_launch(k, dim3(a.g.blocks), dim3(a.g.upb * a.g.tpu), a.g.lds, s, a);
    return hipGetLastError();
}

int ypass_blocks(int ny, int nx) { return ((nx + kYTX - 1) / kYTX) * ((ny + kYTY - 1) / kYTY); }

template <typename T>
hipError_t launch_ypass(const YPassArgs<T>& a, hipStream_t s, int* nblocks) {
    if (a.w > 32) return hipErrorInvalidValue;  // tile slots sized for half-width <= 32
    const size_t lds = (size_t(kYTY + 2 * a.w) * kYTX + size_t(kYTY + 2) * (kYTX + 2)) * sizeof(T);
    dim3 grid((a.nx + kYTX - 1) / kYTX, (a.ny + kYTY - 1) / kYTY);
    if (nblocks) *nblocks = grid.x * grid.y;
    tvd_launch(k_ypass<T>, grid, dim3(kYThreads), lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ypass_full(const YPassArgs<T>& a, hipStream_t s, int* nblocks) {
    if (a.w > kYFMaxH || a.kw > kYFMaxH || a.w < 0 || a.kw < 0) return hipErrorInvalidValue;
    const size_t lds = ypass_full_lds_bytes(a.w, a.kw, sizeof(T));
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ypass_full<T>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    dim3 grid((a.nx + kYTX - 1) / kYTX, (a.ny + kYTY - 1) / kYTY);
    if (nblocks) *nblocks = grid.x * grid.y;
    tvd_launch(k_ypass_full<T>, grid, dim3(kYThreads), lds, s, a);
    return hipGetLastError();
}

template <typename T>
bool mgemm_supported() {
    return true;
}

template <typename T>
hipError_t launch_mgemm(const MGemmArgs<T>& a, hipStream_t s, int* nblocks) {
    const int ts = a.tile == 64 ? 64 : 32;
    dim3 grid((a.N + ts - 1) / ts, (a.M + ts - 1) / ts);
    if (nblocks) *nblocks = int(grid.x * grid.y);
    if (ts == 64) tvd_launch(k_mgemm64<T>, grid, dim3(512), 0, s, a);
    else tvd_launch(k_mgemm<T>, grid, dim3(64 * kMgemmWaves<T>), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mgemm_b(const MGemmArgs<T>* a, int it, BatchGrid g, hipStream_t s) {
    if (g.prefix) {
        if (g.tile == 64) tvd_launch((k_mgemm_bc<T, 64>), dim3(g.total), dim3(256), 0, s, a, it, g.prefix, g.count);
        else tvd_launch((k_mgemm_bc<T, 32>), dim3(g.total), dim3(256), 0, s, a, it, g.prefix, g.count);
        return hipGetLastError();
    }
    if (g.tile == 64) tvd_launch((k_mgemm_b<T, 64>), dim3(g.gx, g.gy, g.count), dim3(256), 0, s, a, it);
    else tvd_launch((k_mgemm_b<T, 32>), dim3(g.gx, g.gy, g.count), dim3(256), 0, s, a, it);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_upd_b(const UpdArgs<T>* a, int it, BatchGrid g, hipStream_t s) {
    tvd_launch(k_upd_b<T>, dim3(g.gx, 1, g.count), dim3(256), 0, s, a, it);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_xpass_b(const XPassArgs<T>* a, BatchGrid g, hipStream_t s) {
    tvd_launch(k_xpass_b<T>, dim3(g.gx, 1, g.count), dim3(256), g.lds, s, a);
    return hipGetLastError();
}

int upd_block_count(int n) { return std::max(1, upd_blocks(n)); }

template <typename T>
hipError_t launch_upd(const UpdArgs<T>& a, hipStream_t s, int* nblocks) {
    const int nb = upd_block_count(a.n);
    if (nblocks) *nblocks = nb;
    tvd_launch(k_upd<T>, dim3(nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// Preconditioned BiCGstab on the reblurring system (van der Vorst 1992):
// the vector stages between the preconditioner solves and the operator
// products (see BcgArgs).  Every block reduces the partials it needs itself
// (the same sums in every block); one thread of the grid records the
// scalars the later stages read.  Each thread owns kBcgE elements (stride
// 256 inside its block's range); its loads are issued before the
// reductions.
// ------------------------------------------------------------------------
constexpr int kBcgE = 4;

int bcg_block_count(int n) { return std::max(1, (n + 256 * kBcgE - 1) / (256 * kBcgE)); }

template <typename T, int kStage>
__global__ void __launch_bounds__(256) k_bcg(BcgArgs<T> a) {
    __shared__ double red[34];
    const int tid = threadIdx.x, bx = blockIdx.x;
    const int base = bx * 256 * kBcgE + tid;
    const bool leader = bx == 0 && tid == 0;
    const int done = a.st->done;
    if constexpr (kStage == 0) {
        double rr = 0.0;
        for (int c = 0; c < kBcgE; ++c) {
            const int k = base + 256 * c;
            if (k >= a.n) continue;
            const T r = a.r[k];
            a.rhat[k] = r;
            a.p[k] = T(0);
            a.v[k] = T(0);
            rr += double(r) * double(r);
        }
        rr = block_sum(rr, red);
        if (tid == 0) {
            a.rr_out[bx] = rr;
            a.rho_out[bx] = rr;
        }
        if (leader) {
            a.sc_st->rho[0] = a.sc_st->rho[1] = 1.0;
            a.sc_st->alpha = a.sc_st->omega = 1.0;
        }
    } else if constexpr (kStage == 1) {
        const double rrp = partial_issue(a.rr_in, a.n_in, tid, 256);
        const double rhp = partial_issue(a.rho_in, a.n_in, tid, 256);
        const double r0 = a.st->r0norm, tol = a.st->tol;
        const int cap = a.st->cap;
        const double rho_old = a.sc_st->rho[(a.iter - 1) & 1];
        const double alpha = a.sc_st->alpha, omega = a.sc_st->omega;
        T rv[kBcgE], pv[kBcgE], vv[kBcgE], sv[kBcgE];
#pragma unroll
        for (int c = 0; c < kBcgE; ++c) {
            const int k = base + 256 * c;
            const bool in = k < a.n;
            rv[c] = in ? a.r[k] : T(0);
            pv[c] = in ? a.p[k] : T(0);
            vv[c] = in ? a.v[k] : T(0);
            sv[c] = (in && a.sc) ? a.sc[k] : T(1);
        }
        if (done) return;
        if (pcg_stop_test(a.st, rrp, a.iter - 1, r0, tol, cap, leader, red)) return;
        const double rho = block_sum(rhp, red);
        if (rho == 0.0 || omega == 0.0) {  // breakdown: keep x of iteration iter - 1
            if (leader) {
                a.st->done = 2;
                a.st->iters = a.iter - 1;
            }
            return;
        }
        const T beta = T((rho / rho_old) * (alpha / omega));
        const T om = T(omega);
#pragma unroll
        for (int c = 0; c < kBcgE; ++c) {
            const int k = base + 256 * c;
            if (k >= a.n) continue;
            const T pn = rv[c] + beta * (pv[c] - om * vv[c]);
            a.p[k] = pn;
            a.tin[k] = sv[c] * pn;
        }
        if (leader) a.sc_st->rho[a.iter & 1] = rho;
    } else if constexpr (kStage == 2) {
        const double sgp = partial_issue(a.sig_in, a.n_y, tid, 256);
        const double rho = a.sc_st->rho[a.iter & 1];
        T rv[kBcgE], vv[kBcgE], sv[kBcgE];
#pragma unroll
        for (int c = 0; c < kBcgE; ++c) {
            const int k = base + 256 * c;
            const bool in = k < a.n;
            rv[c] = in ? a.r[k] : T(0);
            vv[c] = in ? a.v[k] : T(0);
            sv[c] = (in && a.sc) ? a.sc[k] : T(1);
        }
        if (done) return;
        const double sigma = block_sum(sgp, red);
        if (sigma == 0.0) {
            if (leader) {
                a.st->done = 2;
                a.st->iters = a.iter - 1;
            }
            return;
        }
        const double alpha = rho / sigma;
        const T al = T(alpha);
#pragma unroll
        for (int c = 0; c < kBcgE; ++c) {
            const int k = base + 256 * c;
            if (k >= a.n) continue;
            const T sn = rv[c] - al * vv[c];
            a.s[k] = sn;
            a.tin[k] = sv[c] * sn;
        }
        if (leader) a.sc_st->alpha = alpha;
    } else {
        double ts = partial_issue(a.ts_in, a.n_y, tid, 256);
        double tt = partial_issue(a.tt_in, a.n_y, tid, 256);
        const double alpha = a.sc_st->alpha;
        T xv[kBcgE], sv[kBcgE], tv[kBcgE], ph[kBcgE], sh[kBcgE], rh[kBcgE];
#pragma unroll
        for (int c = 0; c < kBcgE; ++c) {
            const int k = base + 256 * c;
            const bool in = k < a.n;
            xv[c] = in ? a.x[k] : T(0);
            sv[c] = in ? a.s[k] : T(0);
            tv[c] = in ? a.t[k] : T(0);
            ph[c] = in ? a.phat[k] : T(0);
            sh[c] = in ? a.shat[k] : T(0);
            rh[c] = in ? a.rhat[k] : T(0);
        }
        if (done) return;
        block_sum2(ts, tt, red);
        const double omega = tt > 0.0 ? ts / tt : 0.0;
        const T al = T(alpha), om = T(omega);
        double rr = 0.0, rhr = 0.0;
#pragma unroll
        for (int c = 0; c < kBcgE; ++c) {
            const int k = base + 256 * c;
            if (k >= a.n) continue;
            a.x[k] = xv[c] + (al * ph[c] + om * sh[c]);
            const T rn = sv[c] - om * tv[c];
            a.r[k] = rn;
            rr += double(rn) * double(rn);
            rhr += double(rh[c]) * double(rn);
        }
        block_sum2(rr, rhr, red);
        if (tid == 0) {
            a.rr_out[bx] = rr;
            a.rho_out[bx] = rhr;
        }
        if (leader) a.sc_st->omega = omega;
    }
}

template <typename T>
hipError_t launch_bcg(const BcgArgs<T>& a, int stage, hipStream_t s, int* nblocks) {
    const int nb = bcg_block_count(a.n);
    if (nblocks) *nblocks = nb;
    switch (stage) {
        case 0: tvd_launch(k_bcg<T, 0>, dim3(nb), dim3(256), 0, s, a); break;
        case 1: tvd_launch(k_bcg<T, 1>, dim3(nb), dim3(256), 0, s, a); break;
        case 2: tvd_launch(k_bcg<T, 2>, dim3(nb), dim3(256), 0, s, a); break;
        case 3: tvd_launch(k_bcg<T, 3>, dim3(nb), dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ypass_full_bcg(const YPassArgs<T>& a, hipStream_t s, int* nblocks) {
    if (a.w > kYFMaxH || a.kw > kYFMaxH || a.w < 0 || a.kw < 0 || !a.dotw || !a.pq_part)
        return hipErrorInvalidValue;
    const size_t lds = ypass_full_lds_bytes(a.w, a.kw, sizeof(T));
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ypass_full_bcg<T>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    dim3 grid((a.nx + kYTX - 1) / kYTX, (a.ny + kYTY - 1) / kYTY);
    if (nblocks) *nblocks = grid.x * grid.y;
    tvd_launch(k_ypass_full_bcg<T>, grid, dim3(kYThreads), lds, s, a);
    return hipGetLastError();
}

// Eigenvalues of AR_2(.) at the two y = 0 frequencies of each axis (first
// and last row and column of the grid) from the interior ones, the end
// eigenvalue of AR(.) being sum_j w_j mu_j (Section 3; level 2 of Section
// 3.2).  The column pass fills the end columns of the interior rows; the row
// pass then fills the end rows over all columns, end columns included, so a
// corner is sum_i wy_i sum_j wx_j lam_ij.  In place: the column pass reads
// only interior entries and the row pass only interior rows.
__global__ void __launch_bounds__(256) k_ar_ext_cols(int ny, int nx, const double* __restrict__ wx, double* l0,
                                                     double* l1, double* l2) {
    __shared__ double red[17];
    double* lam = blockIdx.y == 0 ? l0 : (blockIdx.y == 1 ? l1 : l2);
    if (!lam) return;
    const int i = blockIdx.x + 1;
    double* row = lam + size_t(i) * nx;
    double acc = 0.0;
    for (int j = 1 + int(threadIdx.x); j < nx - 1; j += 256) acc += wx[j - 1] * row[j];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) {
        row[0] = acc;
        row[nx - 1] = acc;
    }
}

// Row pass: a block takes 16 columns; its 16 row groups each sum every 16th
// interior row (independent loads), then one group adds the 16 partials.
constexpr int kArCols = 16, kArGroups = 16;
__global__ void __launch_bounds__(256) k_ar_ext_rows(int ny, int nx, const double* __restrict__ wy, double* l0,
                                                     double* l1, double* l2) {
    __shared__ double part[kArGroups][kArCols + 1];
    double* lam = blockIdx.y == 0 ? l0 : (blockIdx.y == 1 ? l1 : l2);
    if (!lam) return;
    const int c = threadIdx.x % kArCols, g = threadIdx.x / kArCols;
    const int j = blockIdx.x * kArCols + c;
    double acc = 0.0;
    if (j < nx) {
#pragma unroll 8
        for (int i = 1 + g; i < ny - 1; i += kArGroups) acc += wy[i - 1] * lam[size_t(i) * nx + j];
    }
    part[g][c] = acc;
    __syncthreads();
    if (g == 0 && j < nx) {
        double sum = 0.0;
        for (int k = 0; k < kArGroups; ++k) sum += part[k][c];
        lam[j] = sum;
        lam[size_t(ny - 1) * nx + j] = sum;
    }
}

hipError_t launch_ar_extend(int ny, int nx, const double* wy, const double* wx, double* l0, double* l1,
                            double* l2, hipStream_t s) {
    if (ny < 3 || nx < 3) return hipErrorInvalidValue;
    tvd_launch(k_ar_ext_cols, dim3(ny - 2, 3), dim3(256), 0, s, ny, nx, wx, l0, l1, l2);
    tvd_launch(k_ar_ext_rows, dim3((nx + kArCols - 1) / kArCols, 3), dim3(kArCols * kArGroups), 0, s, ny, nx, wy,
               l0, l1, l2);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_xpass(const XPassArgs<T>& a, hipStream_t s) {
    tvd_launch(k_xpass<T>, dim3(a.ny), dim3(256), size_t(a.nx + a.xband_len) * sizeof(T), s, a);
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
    tvd_launch(k_diag_update<T>, dim3(nb), dim3(256), 0, s, n, x, r, p, q, dinv, z, pq_part, n_pq,
                       rz_part, n_rz, rr_out, rz_out, st, iter, do_update, check, rr_in, n_rr_in);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_kappa(int ny, int nx, const T* u, double alpha, double beta, int variant, T* kap,
                        double* kapd, T* s_apply, double* s_mu, double* Dd, hipStream_t s) {
    dim3 grid((nx + 255) / 256, ny);
    tvd_launch(k_kappa<T>, grid, dim3(256), 0, s, ny, nx, u, alpha, beta, variant, kap, kapd, s_apply,
                       s_mu, Dd);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_kappa_ar(int ny, int nx, const T* u, double beta, double* const cdbl[4], T* const cw[4],
                           hipStream_t s) {
    dim3 grid((nx + 255) / 256, ny);
    tvd_launch(k_kappa_ar<T>, grid, dim3(256), 0, s, ny, nx, u, beta, cdbl[0], cdbl[1], cdbl[2], cdbl[3], cw[0],
               cw[1], cw[2], cw[3]);
    return hipGetLastError();
}

hipError_t launch_gemm_operands(int ny, int nx, const double* kapd, const double* s_mu, double* A1,
                                double* A2, double* A3, double* B1, double* B2, double* B3, hipStream_t s) {
    dim3 grid((nx + 255) / 256, ny);
    tvd_launch(k_gemm_operands, grid, dim3(256), 0, s, ny, nx, kapd, s_mu, A1, A2, A3, B1, B2, B3);
    return hipGetLastError();
}

hipError_t launch_gemm(const GemmProblem* probs_dev, int nprob, int maxM, int maxN, hipStream_t s) {
    dim3 grid((maxN + 31) / 32, (maxM + 31) / 32, nprob);
    tvd_launch(k_mgemm_multi, grid, dim3(256), 0, s, probs_dev);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mu(int n, const double* lamh2, const double* lamx, const double* lamy, const double* lamd,
                     int use_lamd, double alpha, double* mu, T* muinv, hipStream_t s) {
    tvd_launch(k_mu<T>, dim3((n + 255) / 256), dim3(256), 0, s, n, lamh2, lamx, lamy, lamd, use_lamd,
                       alpha, mu, muinv);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_objective(int ny, int nx, const double* hu, const T* v, const T* u, double alpha, double beta,
                            double* part, int* nblocks, hipStream_t s) {
    const int nb = std::max(1, std::min(1024, int((size_t(ny) * nx + 255) / 256)));
    *nblocks = nb;
    tvd_launch(k_objective<T>, dim3(nb), dim3(256), 0, s, ny, nx, hu, v, u, alpha, beta, part);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fpchange(int n, const T* x, const T* u, double* part, int* nblocks, hipStream_t s) {
    const int nb = elem_blocks(n, 256, 512);
    *nblocks = nb;
    tvd_launch(k_fpchange<T>, dim3(nb), dim3(256), 0, s, n, x, u, part);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_finalize(PcgState* st, const double* rr_part, int n_rr, const double* fp_part, int n_fp,
                           int max_iter, hipStream_t s) {
    tvd_launch(k_finalize, dim3(1), dim3(256), 0, s, st, rr_part, n_rr, fp_part, n_fp, max_iter);
    return hipGetLastError();
}

hipError_t launch_init_state(PcgState* st, double tol, hipStream_t s) {
    tvd_launch(k_init_state, dim3(1), dim3(1), 0, s, st, tol);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cast_to_double(int n, const T* src, double* dst, hipStream_t s) {
    tvd_launch(k_cast_double<T>, dim3((n + 255) / 256), dim3(256), 0, s, n, src, dst);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_accum(int ny, int nx, const T* lam, const T* hlam, const T* uk1, const double* kapd,
                            double* vbar, double* g, double* part, int* nblocks, hipStream_t s) {
    const int nb = elem_blocks(ny * nx, 256, 1024);
    *nblocks = nb;
    tvd_launch(k_adj_accum<T>, dim3(nb), dim3(256), 0, s, ny, nx, lam, hlam, uk1, kapd, vbar, g, part);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_ubar(int ny, int nx, const double* g, const T* uk, double alpha, double* ubar, hipStream_t s) {
    const int nb = elem_blocks(ny * nx, 256, 2048);
    tvd_launch(k_adj_ubar<T>, dim3(nb), dim3(256), 0, s, ny, nx, g, uk, alpha, ubar);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cast_from_double(int n, const double* src, T* dst, hipStream_t s) {
    tvd_launch(k_cast_from_double<T>, dim3((n + 255) / 256), dim3(256), 0, s, n, src, dst);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_add_to_double(int n, const T* src, double* dst, hipStream_t s) {
    tvd_launch(k_add_to_double<T>, dim3((n + 255) / 256), dim3(256), 0, s, n, src, dst);
    return hipGetLastError();
}

template <typename T>
LineGeom line_geom_block(int lines, int n, int M, int threads) {
    LineGeom g{};
    g.units = (lines + 1) / 2;
    // same threads-per-pair rule as line_geom, capped by the block size;
    // the block then holds threads / tpu pairs so that every lane has a pair
    int tpu = std::min(256, std::max(64, M / 8));
    while (tpu < n && tpu < 1024) tpu *= 2;
    tpu = std::min(tpu, threads);
    if (tpu * kLinePos < n || threads % tpu != 0) return LineGeom{};
    g.tpu = tpu;
    g.upb = threads / tpu;
    g.blocks = (g.units + g.upb - 1) / g.upb;
    g.lds = size_t(2) * padded_len(M) * sizeof(cx<T>) * g.upb;
    return g;
}

size_t ypass_lds_bytes(int w, size_t elem) {
    return (size_t(kYTY + 2 * w) * kYTX + size_t(kYTY + 2) * (kYTX + 2)) * elem;
}
size_t ypass_full_lds_bytes(int wy, int wx, size_t elem) {
    const size_t tw = kYTX + 2 * std::max(wx, 1);
    return (size_t(kYTY + 2 * std::max(wy, 1)) * tw + size_t(kYTY) * tw) * elem;
}

static void allow_lds(const void* k, size_t lds) {
    if (lds > 64 * 1024) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
}

template <typename T>
hipError_t launch_kappa_b(const KappaArgs<T>* a, BatchGrid g, hipStream_t s) {
    tvd_launch(k_kappa_b<T>, dim3(g.gx, g.gy, g.count), dim3(256), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_operands_b(const OperandArgs* a, BatchGrid g, hipStream_t s) {
    tvd_launch(k_operands_b, dim3(g.gx, g.gy, g.count), dim3(256), 0, s, a);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_mu_b(const MuArgs<T>* a, BatchGrid g, hipStream_t s) {
    tvd_launch(k_mu_b<T>, dim3(g.gx, 1, g.count), dim3(256), 0, s, a);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_fpchange_b(const FpArgs<T>* a, BatchGrid g, hipStream_t s) {
    tvd_launch(k_fpchange_b<T>, dim3(g.gx, 1, g.count), dim3(256), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_finalize_b(const FinArgs* a, int count, hipStream_t s) {
    tvd_launch(k_finalize_b, dim3(count), dim3(256), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_init_b(const InitArgs* a, int count, hipStream_t s) {
    tvd_launch(k_init_b, dim3(count), dim3(64), 0, s, a);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_copy_b(const CopyArgs<T>* a, BatchGrid g, hipStream_t s) {
    tvd_launch(k_copy_b<T>, dim3(g.gx, 1, g.count), dim3(256), 0, s, a);
    return hipGetLastError();
}
template <typename TX, typename TS, typename TA, typename TY>
hipError_t launch_band_b(const BandArgsT<TX, TS, TA, TY>* a, BatchGrid g, hipStream_t s) {
    allow_lds(reinterpret_cast<const void*>(&k_band_b<TX, TS, TA, TY>), g.lds);
    tvd_launch((k_band_b<TX, TS, TA, TY>), dim3(g.gx, g.gy, g.count), dim3(kBandThreads), g.lds, s, a);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_rowpass_b(const RowPassArgs<T>* a, int it, bool tab_lds, BatchGrid g, hipStream_t s) {
    auto k = tab_lds ? &k_rowpass_b<T, true> : &k_rowpass_b<T, false>;
    allow_lds(reinterpret_cast<const void*>(k), g.lds);
    tvd_launch(k, dim3(g.gx, 1, g.count), dim3(g.threads), g.lds, s, a, it);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_colpass_b(const ColPassArgs<T>* a, int it, bool tab_lds, BatchGrid g, hipStream_t s) {
    auto k = tab_lds ? &k_colpass_b<T, true> : &k_colpass_b<T, false>;
    allow_lds(reinterpret_cast<const void*>(k), g.lds);
    tvd_launch(k, dim3(g.gx, 1, g.count), dim3(g.threads), g.lds, s, a, it);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_ypass_b(const YPassArgs<T>* a, BatchGrid g, hipStream_t s) {
    allow_lds(reinterpret_cast<const void*>(&k_ypass_b<T>), g.lds);
    tvd_launch(k_ypass_b<T>, dim3(g.gx, g.gy, g.count), dim3(kYThreads), g.lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ypass_full_b(const YPassArgs<T>* a, BatchGrid g, hipStream_t s) {
    if (g.prefix) {
        allow_lds(reinterpret_cast<const void*>(&k_ypass_full_bc<T>), g.lds);
        tvd_launch(k_ypass_full_bc<T>, dim3(g.total), dim3(kYThreads), g.lds, s, a, g.prefix, g.count);
        return hipGetLastError();
    }
    allow_lds(reinterpret_cast<const void*>(&k_ypass_full_b<T>), g.lds);
    tvd_launch(k_ypass_full_b<T>, dim3(g.gx, g.gy, g.count), dim3(kYThreads), g.lds, s, a);
    return hipGetLastError();
}

#define TVD_INSTANTIATE(T)                                                                                    \
    template bool mgemm_supported<T>();                                                                       \
    template hipError_t launch_mgemm<T>(const MGemmArgs<T>&, hipStream_t, int*);                              \
    template hipError_t launch_upd<T>(const UpdArgs<T>&, hipStream_t, int*);                                  \
    template hipError_t launch_bcg<T>(const BcgArgs<T>&, int, hipStream_t, int*);                             \
    template hipError_t launch_ypass_full_bcg<T>(const YPassArgs<T>&, hipStream_t, int*);                     \
    template hipError_t launch_mgemm_b<T>(const MGemmArgs<T>*, int, BatchGrid, hipStream_t);                  \
    template hipError_t launch_upd_b<T>(const UpdArgs<T>*, int, BatchGrid, hipStream_t);                      \
    template hipError_t launch_xpass_b<T>(const XPassArgs<T>*, BatchGrid, hipStream_t);                       \
    template hipError_t launch_xpass<T>(const XPassArgs<T>&, hipStream_t);                                    \
    template hipError_t launch_kappa_b<T>(const KappaArgs<T>*, BatchGrid, hipStream_t);                       \
    template hipError_t launch_mu_b<T>(const MuArgs<T>*, BatchGrid, hipStream_t);                             \
    template hipError_t launch_fpchange_b<T>(const FpArgs<T>*, BatchGrid, hipStream_t);                       \
    template hipError_t launch_copy_b<T>(const CopyArgs<T>*, BatchGrid, hipStream_t);                         \
    template hipError_t launch_band_b<T, T, double, T>(const BandArgsT<T, T, double, T>*, BatchGrid,          \
                                                       hipStream_t);                                          \
    template hipError_t launch_rowpass_b<T>(const RowPassArgs<T>*, int, bool, BatchGrid, hipStream_t);        \
    template hipError_t launch_colpass_b<T>(const ColPassArgs<T>*, int, bool, BatchGrid, hipStream_t);        \
    template hipError_t launch_ypass_b<T>(const YPassArgs<T>*, BatchGrid, hipStream_t);                       \
    template hipError_t launch_ypass_full_b<T>(const YPassArgs<T>*, BatchGrid, hipStream_t);                  \
    template LineGeom line_geom_block<T>(int, int, int, int);                                                 \
    template hipError_t launch_adj_accum<T>(int, int, const T*, const T*, const T*, const double*, double*,   \
                                            double*, double*, int*, hipStream_t);                             \
    template hipError_t launch_adj_ubar<T>(int, int, const double*, const T*, double, double*, hipStream_t);  \
    template hipError_t launch_cast_from_double<T>(int, const double*, T*, hipStream_t);                      \
    template hipError_t launch_add_to_double<T>(int, const T*, double*, hipStream_t);                         \
    template hipError_t launch_band<T, T, T, T>(const BandArgs<T>&, int, hipStream_t, int*);                  \
    template size_t band_lds_bytes<T, T, T, T>(const BandArgs<T>&, int);                                      \
    template LineGeom line_geom<T>(int, int, int);                                                            \
    template size_t lds_table_bytes<T>(int);                                                                  \
    template hipError_t launch_rowpass<T>(const RowPassArgs<T>&, hipStream_t);                                \
    template hipError_t launch_ypass<T>(const YPassArgs<T>&, hipStream_t, int*);                              \
    template hipError_t launch_ypass_full<T>(const YPassArgs<T>&, hipStream_t, int*);                         \
    template hipError_t launch_colpass<T>(const ColPassArgs<T>&, hipStream_t);                                \
    template hipError_t launch_diag_update<T>(int, T*, T*, const T*, const T*, const T*, T*, const double*,   \
                                              int, const double*, int, double*, double*, PcgState*, int, int, \
                                              int, const double*, int, int*, hipStream_t);                    \
    template hipError_t launch_kappa<T>(int, int, const T*, double, double, int, T*, double*, T*, double*,    \
                                        double*, hipStream_t);                                                \
    template hipError_t launch_kappa_ar<T>(int, int, const T*, double, double* const[4], T* const[4],         \
                                           hipStream_t);                                                      \
    template hipError_t launch_objective<T>(int, int, const double*, const T*, const T*, double, double,      \
                                            double*, int*, hipStream_t);                                      \
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

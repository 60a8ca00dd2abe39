// Internal interfaces of libtvdeblur: device-side argument blocks shared by
// the host driver (tvd_capi.cpp) and the kernels (tvd_kernels.hip), and the
// host-side precomputation routines (tvd_plan.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace tvd {

template <typename T>
struct cx {
    T x, y;
};

// PCG control block, one per solve, in device memory.  Written only by
// block 0 of a kernel; read by later kernels on the same stream.
struct PcgState {
    double r0norm;     // ||r_0||
    double tol;        // inner tolerance
    double relres;     // ||r_i|| / ||r_0|| at the last convergence test
    double fp_change;  // ||x - u|| / ||x||, filled by the step finaliser
    int done;          // 0 running, 1 converged, 2 breakdown, 3 no steps this solve
    int iters;         // iterations completed when done != 0
    int cap;           // > 0: stop after exactly this many iterations (replay)
    int pad;
};

// Transform plan for one axis: 1D DST-I on the interior (anti-reflective)
// or DCT-II / DCT-III (reflective), computed two image lines at a time as
// one complex DFT of length L (Stockham radix-2 when L is a power of two,
// Bluestein through a power-of-two M otherwise).
template <typename T>
struct AxisPlan {
    int n;          // line length
    int kind;       // 1 = DST-I interior (AR), 2 = DCT-II/III (reflective)
    int L, M, log2M, bluestein;
    const cx<T>* tw;     // M twiddles exp(-2 pi i t / M)
    const cx<T>* chirp;  // L entries exp(-i pi t^2 / L)      (Bluestein)
    const cx<T>* bf;     // M entries FFT_M(conj chirp, wrapped) / M (Bluestein)
    const cx<T>* pre;    // n entries: DCT-III input weights w_k exp(+i pi k/(2n))
    const cx<T>* post;   // n entries: DCT-II output weights w_k exp(-i pi k/(2n)) / 2
    T dst_scale;         // 1/sqrt(2(n-1))
    // All tables above, contiguous in one device blob (tw | chirp | bf | pre |
    // post, each padded to an even count) so a block can copy them into LDS
    // with 16-byte loads; offsets in complex entries.
    const cx<T>* blob;
    int blob_len;        // even
    int off_chirp, off_bf, off_pre, off_post;
    int tables_in_lds;   // copy the blob into LDS (if it fits next to the FFT buffers)
};

// Launch geometry of a line pass.
struct LineGeom {
    int units;   // line pairs
    int upb;     // units per block
    int tpu;     // threads per unit
    int blocks;
    size_t lds;  // dynamic LDS bytes
};

// Banded Kronecker operator  Y = sum_r (By_r (x) Bx_r) X  (+ alpha L(S) X,
// optional p-update of the input, residual form and FP64 dot partials).
// TX: band input (and p-update) storage, TS: separate stencil input storage,
// TA: band coefficients, diffusivity, residual right-hand side and the
// accumulation type, TY: output storage.
template <typename TX, typename TS, typename TA, typename TY>
struct BandArgsT {
    int ny, nx;
    int wy, wx, nterms;
    const TA* By;          // [nterms][ny][2wy+1]
    const TA* Bx;          // [nterms][nx][2wx+1]
    const TX* X;           // input, or p_old when Z != nullptr
    const TX* Z;           // p-update: X_eff = Z + beta X
    TX* Xnew;              // receives X_eff (own tile) when Z != nullptr
    const double* rz_new;  // beta = sum(rz_new)/sum(rz_old); rz_old == nullptr -> beta = 0
    const double* rz_old;
    int n_rz;
    const TA* kap;         // stencil diffusivity (nullptr: no stencil)
    double alpha;
    const TS* S;           // stencil input; nullptr -> the (updated) band input
    const TA* Bvec;        // residual form Y = Bvec - result when non-null
    TY* Y;
    double* dot_part;      // per-block partials
    int dotmode;           // 0 none, 1 <stencil input, result>, 2 <Y, Y>,
                           // 3 <W, Y> (and <Y, Y> into dot_part2 when set)
    const TS* W;
    double* dot_part2;
    const PcgState* st;    // exit when st->done (nullable)
    int tile_y;            // tile height (8 or 16), chosen by the launcher
    int bgx, bgy;          // this image's grid (set by the launcher; batched launches)
    int wrap;              // periodic BCs: the input wraps around (circulant bands)
    const TA* cst;         // nullptr, or 4 N per-pixel stencil coefficients (up, down,
                           // left, right; the anti-reflective L) used instead of kap
};
template <typename T>
using BandArgs = BandArgsT<T, T, T, T>;

template <typename T>
struct RowPassArgs {
    int ny, nx;
    AxisPlan<T> plan;       // along rows (length nx)
    LineGeom g;
    int mode;               // 0 forward (s o r -> T1), 1 inverse (T2 -> z = s o ., <r,z>)
    int do_update;          // mode 0: x += a p, r -= a q first; a = sum(rz)/sum(pq)
    T* x;
    T* r;
    const T* p;
    const T* q;
    const double* pq_part;
    int n_pq;
    const double* rz_part;
    int n_rz;
    const T* s;             // scaling (nullptr = 1)
    const T* src;
    T* dst;
    double* part_out;       // mode 0: ||r||^2 partials, mode 1: <r,z> partials
    PcgState* st;
    int iter;
    // mode 1 only: also w = (I (x) K_x) z along the rows held in LDS.
    // K_x is Toeplitz on rows [klo, khi); xband = [Toeplitz row | rows < klo
    // | rows >= khi], each 2*kw+1 wide, copied to LDS (xband_len reals).
    T* wout;                // nullptr: no x-pass
    const T* xband;
    int kw, klo, khi, xband_len;
    // 1: the transform is T_n of the anti-reflective algebra instead of S^
    // (DST-I plans only): mode 0 applies T_n^{-1} (the interior minus the
    // linear interpolant of the two end values, then S^), mode 1 applies
    // T_n (S^, then the interior plus that interpolant)
    int ramp;
};

// Column half of the fused normal operator for the PCG direction update:
// tmp_new = w + beta tmp_old, p_new = z + beta p_old (own tile written),
// q = (K_y (x) I) tmp_new + alpha L(u^k) p_new, <p_new, q> partials.
template <typename T>
struct YPassArgs {
    int ny, nx, w;
    const T* Ky;            // [ny][2w+1]
    const T* wv;            // (I (x) K_x) z of this iteration
    const T* tmp_old;
    T* tmp_new;
    const T* z;
    const T* p_old;
    T* p_new;
    const T* kap;
    double alpha;
    const double* rz_new;   // beta = sum(rz_new)/sum(rz_old); rz_old == nullptr -> beta = 0
    const double* rz_old;
    int n_rz;
    T* q;
    double* pq_part;
    const PcgState* st;
    // whole-operator form (k_ypass_full): the row band, Toeplitz-compressed
    // (interior row, then rows 0..klo-1, then rows khi..nx-1), half-width kw
    const T* xband;
    int kw, klo, khi;
    // BiCGstab form (k_ypass_full_bcg): beta = 0, no p copy; the partials
    // are <dotw, q> into pq_part and, when qq_part is set, <q, q> into it
    const T* dotw;
    double* qq_part;
    int wrap;               // periodic BCs: tile halos wrap around (circulant bands)
    const T* cst;           // BiCGstab form: nullptr, or 4 N per-pixel stencil
                            // coefficients (the anti-reflective L) instead of kap
};

// Scalars of preconditioned BiCGstab carried between its launches: rho by
// iteration parity (written by the direction stage of iteration i into
// rho[i & 1], read as rho_old by iteration i + 1), alpha and omega of the
// last completed stages.
struct BcgScalars {
    double rho[2];
    double alpha;
    double omega;
};

// Vector stages of BiCGstab on the reblurring system (k_bcg):
//   0 init:      rhat = r, p = v = 0; partials ||r||^2, <rhat, r>; scalars 1
//   1 direction: stopping test on ||r_{i-1}||, rho = <rhat, r_{i-1}>,
//                p = r + beta (p - omega v), tin = sc o p
//   2 s-update:  alpha = rho / <rhat, v>, s = r - alpha v, tin = sc o s
//   3 x-update:  omega = <t, s> / <t, t>, x += alpha phat + omega shat,
//                r = s - omega t; partials ||r||^2, <rhat, r>
template <typename T>
struct BcgArgs {
    int n;
    int iter;
    T* x;
    T* r;
    T* rhat;
    T* p;
    T* v;
    T* s;
    const T* t;
    const T* phat;
    const T* shat;
    const T* sc;            // D^{-1/2} of D_P / P_D; nullptr: ones
    T* tin;                 // preconditioner input
    const double* rr_in;    // stage 1: ||r||^2 and <rhat, r> partials
    const double* rho_in;
    int n_in;
    const double* sig_in;   // stage 2: <rhat, v> partials
    const double* ts_in;    // stage 3: <t, s> and <t, t> partials
    const double* tt_in;
    int n_y;                // partials of stages 2 and 3 (y-pass blocks)
    double* rr_out;         // stages 0 and 3
    double* rho_out;
    BcgScalars* sc_st;
    PcgState* st;
};

// Dense product on the matrix cores, C = A Bt^T: A is M x K and Bt is N x K,
// both row-major (k contiguous); C is M x N row-major, or stored transposed
// (N x M row-major) with transC.  An optional PCG stopping test runs before
// the product and an elementwise epilogue after it (on the M x N layout).
template <typename T>
struct MGemmArgs {
    int M, N, K;
    const T* A;
    const T* Bt;
    T* C;
    int transC;
    int epi;                // 0: C = AB; 1: C = E1 o AB; 2: C = E1 o AB and <E2, C> partials
    const T* E1;
    const T* E2;
    double* part;           // epi 2: one partial per block (by * gridDim.x + bx)
    int check;              // stopping test from rr partials (as the column pass)
    const double* rr_part;
    int n_rr;
    int iter;
    PcgState* st;           // nullptr: plain product
    int tile;               // block tile: 32 (four waves, eight in FP64, split K
                            // of one 32 x 32 tile) or 64 (64 x 64, one 32 x 32
                            // quadrant per wave; single image: two groups of
                            // four waves split K)
};

// PCG update of the product-form preconditioner path: x += a p, r -= a q
// (a from the <p, q> and <r, z> partials), ||r||^2 partials, and the
// preconditioner input t = s o r (or r).  do_update = 0: t only.
template <typename T>
struct UpdArgs {
    int n;
    int do_update;
    T* x;
    T* r;
    const T* p;
    const T* q;
    const T* s;
    T* t;
    const double* pq_part;
    int n_pq;
    const double* rz_part;
    int n_rz;
    double* rr_out;
    PcgState* st;
    int iter;
};

// Row half of the fused normal operator on its own: w = (I (x) K_x) z with
// the Toeplitz-compressed band (see compress_band).
template <typename T>
struct XPassArgs {
    int ny, nx;
    const T* z;
    T* w;
    const T* xband;
    int xband_len;
    int kw, klo, khi;
    const PcgState* st;
};

template <typename T>
struct ColPassArgs {
    int ny, nx;
    AxisPlan<T> plan;       // along columns (length ny)
    LineGeom g;
    const T* src;
    T* dst;
    const T* muinv;
    int check;              // convergence test from rr partials before work
    const double* rr_part;
    int n_rr;
    PcgState* st;
    int iter;
    int ramp;               // 1: T_n^{-1}, then T_n along the columns (see RowPassArgs)
};

// FP64 GEMM problem C = sum_t coef_t op(A_t) B_t (row-major).
struct GemmTerm {
    const double* A;
    const double* B;
    double coef;
};
struct GemmProblem {
    int M, N, K;
    int transA;
    int nterms;
    GemmTerm t[3];
    double* C;
};

// Per-image argument blocks of the small per-step kernels (batched launches).
template <typename T>
struct KappaArgs {
    int ny, nx;
    const T* u;
    double alpha, beta;
    int variant;
    T* kap;
    double* kapd;
    T* s_apply;
    double* s_mu;
    double* Dd;
};
struct OperandArgs {
    int ny, nx;
    const double* kapd;
    const double* s_mu;
    double *A1, *A2, *A3, *B1, *B2, *B3;
};
template <typename T>
struct MuArgs {
    int n;
    const double *lamh2, *lamx, *lamy, *lamd;
    int use_lamd;
    double alpha;
    double* mu;
    T* muinv;
};
template <typename T>
struct FpArgs {
    int n, nb;
    const T* x;
    const T* u;
    double* part;
};
struct FinArgs {
    PcgState* st;
    const double* rr_part;
    int n_rr;
    const double* fp_part;
    int n_fp;
    int max_iter;
};
struct InitArgs {
    PcgState* st;
    double tol;
    int frozen;  // nonzero: the image takes no PCG steps (done = 3)
    int cap;     // PcgState::cap
};
template <typename T>
struct CopyArgs {
    int n;
    const T* src;
    T* dst;
};

// Batched launches: one kernel per stage for all images of a batch
// (image = blockIdx.z, argument blocks in device memory).
struct BatchGrid {
    int gx, gy, count;
    size_t lds;
    int threads;
    int tile;  // batched products: block tile (32 or 64)
    // compact grids: blocks [prefix[i], prefix[i+1]) belong to image i and
    // the launch has prefix[count] blocks (nullptr: gx x gy x count grid)
    const int* prefix;
    int total;
};
template <typename T>
hipError_t launch_kappa_b(const KappaArgs<T>* a, BatchGrid g, hipStream_t s);
hipError_t launch_operands_b(const OperandArgs* a, BatchGrid g, hipStream_t s);
template <typename T>
hipError_t launch_mu_b(const MuArgs<T>* a, BatchGrid g, hipStream_t s);
template <typename T>
hipError_t launch_fpchange_b(const FpArgs<T>* a, BatchGrid g, hipStream_t s);
hipError_t launch_finalize_b(const FinArgs* a, int count, hipStream_t s);
hipError_t launch_init_b(const InitArgs* a, int count, hipStream_t s);
template <typename T>
hipError_t launch_copy_b(const CopyArgs<T>* a, BatchGrid g, hipStream_t s);
template <typename TX, typename TS, typename TA, typename TY>
hipError_t launch_band_b(const BandArgsT<TX, TS, TA, TY>* a, BatchGrid g, hipStream_t s);
template <typename T>
hipError_t launch_rowpass_b(const RowPassArgs<T>* a, int it, bool tab_lds, BatchGrid g, hipStream_t s);
template <typename T>
hipError_t launch_colpass_b(const ColPassArgs<T>* a, int it, bool tab_lds, BatchGrid g, hipStream_t s);
template <typename T>
hipError_t launch_ypass_b(const YPassArgs<T>* a, BatchGrid g, hipStream_t s);
template <typename T>
hipError_t launch_ypass_full_b(const YPassArgs<T>* a, BatchGrid g, hipStream_t s);
// Line geometry for a batched pass whose blocks all have `threads` threads
// (tpu = 0 if a line does not fit).
template <typename T>
LineGeom line_geom_block(int lines, int n, int M, int threads);
size_t ypass_lds_bytes(int w, size_t elem);
size_t ypass_full_lds_bytes(int wy, int wx, size_t elem);

// Arm a start/stop event pair for the next kernel launch of this thread;
// disarm returns whether a launch consumed them.
void arm_kernel_events(hipEvent_t start, hipEvent_t stop);
bool disarm_kernel_events();

// ---- kernel launchers (tvd_kernels.hip) ----
// Launch with tile height ty (8 or 16); band_lds_bytes gives the dynamic
// LDS the launch needs, band_blocks the grid size (= number of partials).
template <typename TX, typename TS, typename TA, typename TY>
hipError_t launch_band(const BandArgsT<TX, TS, TA, TY>& a, int ty, hipStream_t s, int* nblocks_out);
int band_blocks(int ny, int nx, int ty);
template <typename TX, typename TS, typename TA, typename TY>
size_t band_lds_bytes(const BandArgsT<TX, TS, TA, TY>& a, int ty);
template <typename T>
hipError_t launch_rowpass(const RowPassArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_ypass(const YPassArgs<T>& a, hipStream_t s, int* nblocks);
template <typename T>
hipError_t launch_ypass_full(const YPassArgs<T>& a, hipStream_t s, int* nblocks);
template <typename T>
hipError_t launch_ypass_full_bcg(const YPassArgs<T>& a, hipStream_t s, int* nblocks);
template <typename T>
hipError_t launch_bcg(const BcgArgs<T>& a, int stage, hipStream_t s, int* nblocks);
// In place: end rows / columns of up to three ny x nx eigenvalue arrays
// (nullptr skipped) from their interior with the end weights wy, wx.
hipError_t launch_ar_extend(int ny, int nx, const double* wy, const double* wx, double* l0, double* l1,
                            double* l2, hipStream_t s);
// Matrix-core product; *nblocks = number of blocks (= partials of epi 2).
// Only for element types whose MFMA layout is supported (mgemm_supported).
template <typename T>
hipError_t launch_mgemm(const MGemmArgs<T>& a, hipStream_t s, int* nblocks);
template <typename T>
bool mgemm_supported();
template <typename T>
hipError_t launch_upd(const UpdArgs<T>& a, hipStream_t s, int* nblocks);
template <typename T>
hipError_t launch_xpass(const XPassArgs<T>& a, hipStream_t s);
// Batched product-form kernels (image = blockIdx.z; see BatchGrid).
template <typename T>
hipError_t launch_mgemm_b(const MGemmArgs<T>* a, int it, BatchGrid g, hipStream_t s);
template <typename T>
hipError_t launch_upd_b(const UpdArgs<T>* a, int it, BatchGrid g, hipStream_t s);
template <typename T>
hipError_t launch_xpass_b(const XPassArgs<T>* a, BatchGrid g, hipStream_t s);
int upd_block_count(int n);
int bcg_block_count(int n);
int ypass_blocks(int ny, int nx);
template <typename T>
hipError_t launch_colpass(const ColPassArgs<T>& a, hipStream_t s);
template <typename T>
LineGeom line_geom(int lines, int n, int M);
// LDS bytes reserved for a plan's table blob of blob_len complex entries.
template <typename T>
size_t lds_table_bytes(int blob_len);

template <typename T>
hipError_t launch_diag_update(int n, T* x, T* r, const T* p, const T* q, const T* dinv, T* z,
                              const double* pq_part, int n_pq, const double* rz_part, int n_rz,
                              double* rr_out, double* rz_out, PcgState* st, int iter, int do_update,
                              int check, const double* rr_in, int n_rr_in, int* nblocks, hipStream_t s);

template <typename T>
hipError_t launch_kappa_ar(int ny, int nx, const T* u, double beta, double* const cdbl[4], T* const cw[4],
                           hipStream_t s);
template <typename T>
hipError_t launch_objective(int ny, int nx, const double* hu, const T* v, const T* u, double alpha, double beta,
                            double* part, int* nblocks, hipStream_t s);
template <typename T>
hipError_t launch_kappa(int ny, int nx, const T* u, double alpha, double beta, int variant,
                        T* kap, double* kapd, T* s_apply, double* s_mu, double* Dd, hipStream_t s);
hipError_t launch_gemm_operands(int ny, int nx, const double* kapd, const double* s_mu, double* A1,
                                double* A2, double* A3, double* B1, double* B2, double* B3,
                                hipStream_t s);
hipError_t launch_gemm(const GemmProblem* probs_dev, int nprob, int maxM, int maxN, hipStream_t s);
template <typename T>
hipError_t launch_mu(int n, const double* lamh2, const double* lamx, const double* lamy,
                     const double* lamd, int use_lamd, double alpha, double* mu, T* muinv,
                     hipStream_t s);
template <typename T>
hipError_t launch_fpchange(int n, const T* x, const T* u, double* part, int* nblocks, hipStream_t s);
template <typename T>
hipError_t launch_finalize(PcgState* st, const double* rr_part, int n_rr, const double* fp_part,
                           int n_fp, int max_iter, hipStream_t s);
template <typename T>
hipError_t launch_cast_to_double(int n, const T* src, double* dst, hipStream_t s);
hipError_t launch_init_state(PcgState* st, double tol, hipStream_t s);
// Adjoint step pieces (differentiation form).
template <typename T>
hipError_t launch_adj_accum(int ny, int nx, const T* lam, const T* hlam, const T* uk1, const double* kapd,
                            double* vbar, double* g, double* part, int* nblocks, hipStream_t s);
template <typename T>
hipError_t launch_adj_ubar(int ny, int nx, const double* g, const T* uk, double alpha, double* ubar,
                           hipStream_t s);
template <typename T>
hipError_t launch_cast_from_double(int n, const double* src, T* dst, hipStream_t s);
template <typename T>
hipError_t launch_add_to_double(int n, const T* src, double* dst, hipStream_t s);

// ---- host precomputation (tvd_plan.cpp) ----
struct PsfFactors {
    int my, mx, rank;
    std::vector<std::vector<double>> gy, gx;  // rank terms; h ~ sum gy_r gx_r^T
};
int validate_psf(const double* h, int py, int px, std::string& err);
PsfFactors factor_psf(const double* h, int py, int px);

// Dense 1D blur matrix (n x n, row-major) of the 1D filter g (length 2m+1,
// centre at m) under the boundary condition bc (1 reflective, 2 AR, 3 zero
// Dirichlet, 4 periodic).
std::vector<double> blur_matrix_1d(const std::vector<double>& g, int n, int bc);
// Band of a dense n x n matrix: out[i*(2w+1) + d + w] = A[i][i+d] (0 outside).
std::vector<double> band_of(const std::vector<double>& A, int n, int w);
// Band of a circulant n x n matrix: out[i*(2w+1) + d + w] = A[i][(i+d) mod n]
// (2w + 1 <= n, so no entry is counted twice).
std::vector<double> band_wrapped(const std::vector<double>& A, int n, int w);
std::vector<double> transpose(const std::vector<double>& A, int n);
// Band rows [lo, hi) all equal one Toeplitz row; data = [that row | rows < lo
// | rows >= hi], each 2w+1 wide (lo = hi = n when no row repeats).
struct ToeplitzBand {
    int w, lo, hi;
    std::vector<double> data;
};
ToeplitzBand compress_band(const std::vector<double>& band, int n, int w);
std::vector<double> matmul_tn(const std::vector<double>& A, const std::vector<double>& B, int n);

// Basis matrix Phi[i*n + k] = phi_k(i) of the transform of the BC (DCT-II
// for reflective and zero-Dirichlet, S^ for AR, the real Fourier basis for
// periodic).
std::vector<double> basis_matrix(int n, int bc);
// lambda_H[k*nx + l] = h^(theta_k, theta_l) on the BC grid; for zero
// Dirichlet the optimal cosine-algebra projection diag(Q2 H Q2^T).
std::vector<double> symbol_eigenvalues(const double* h, int py, int px, int ny, int nx, int bc);
// T_n and T_n^{-1} of the anti-reflective algebra, row-major (n >= 3).
void ar_transform_matrices(int n, std::vector<double>& T, std::vector<double>& Ti);
// n - 2 weights w: the end eigenvalue of AR(A) is sum_j w_j mu_j over the
// interior eigenvalues mu of s(A_in).
std::vector<double> ar_end_weights(int n);

struct AxisTables {
    int n, kind, L, M, log2M, bluestein;
    std::vector<double> tw, chirp, bf, pre, post;  // interleaved re, im
    double dst_scale;
    // tw | chirp | bf | pre | post, each padded to an even number of entries
    std::vector<double> blob;
    int off_chirp, off_bf, off_pre, off_post, blob_len;
};
AxisTables make_axis_tables(int n, int bc);

}  // namespace tvd

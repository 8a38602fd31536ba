// Shared device/host definitions for libmpo (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "profiler.h"

namespace mpo {

// Interleaved complex value of the working precision (double2 / float2).
template <typename T> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename T> using C2 = typename cvec<T>::type;

// 4-wide accumulator of one 16x16x4 MFMA (one lane's share of a 16x16 tile).
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
template <typename T> struct accv;
template <> struct accv<double> { using type = d4; };
template <> struct accv<float> { using type = f4; };
template <typename T> using A4 = typename accv<T>::type;

// D(16x16) += A(16x4) * B(4x16).  Operand layout (wave64): lane l supplies
// A[l%16][l/16] and B[l/16][l%16].  Result element r of lane l is
// D[acc_row<T>(l, r)][l%16]: rows 4*(l/16)+r for f32, but interleaved rows
// (l/16)+4*r for f64 (both checked on gfx950).
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------ split-BF16x3
// An FP32 value x is carried as hi + lo with hi = bf16(x) and lo = bf16(x - hi)
// (round to nearest even; x - hi is exact in FP32), i.e. about 16 significant
// bits.  A real product a*b is taken as ah*bh + ah*bl + al*bh (the al*bl term,
// of relative size 2^-16, is dropped) on the BF16 MFMA with FP32 accumulation.
// v_mfma_f32_16x16x16_bf16 layout (wave64, checked on gfx950): lane l supplies
// A[l%16][4(l/16)+j] and B[4(l/16)+j][l%16], j = 0..3; the result layout is
// that of the FP32 16x16x4 product.
typedef short bf4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned bf16_bits(float x) {
    const unsigned u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// Four complex FP32 values (k = 0..3 of one row or column) as BF16 hi/lo parts
// of the real and imaginary components; conj negates the imaginary parts.
struct CBF { bf4 rh, rl, ih, il; };

__device__ __forceinline__ CBF cbf_split(const float2 (&v)[4], bool conj) {
    CBF o;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float re = v[j].x, im = conj ? -v[j].y : v[j].y;
        const unsigned rh = bf16_bits(re), ih = bf16_bits(im);
        o.rh[j] = (short)rh;
        o.ih[j] = (short)ih;
        o.rl[j] = (short)bf16_bits(re - __uint_as_float(rh << 16));
        o.il[j] = (short)bf16_bits(im - __uint_as_float(ih << 16));
    }
    return o;
}

__device__ __forceinline__ f4 mfma_bf16(bf4 a, bf4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// (accR, accI) += A * B for one 16x16x16 complex tile product, 12 BF16 MFMAs.
__device__ __forceinline__ void cmfma_bf3(f4& accR, f4& accI, const CBF& a, const CBF& b) {
    const bf4 sign = {(short)0x8000, (short)0x8000, (short)0x8000, (short)0x8000};
    const bf4 nih = a.ih ^ sign, nil = a.il ^ sign;
    accR = mfma_bf16(a.rl, b.rh, accR);
    accR = mfma_bf16(a.rh, b.rl, accR);
    accR = mfma_bf16(nil, b.ih, accR);
    accR = mfma_bf16(nih, b.il, accR);
    accR = mfma_bf16(a.rh, b.rh, accR);
    accR = mfma_bf16(nih, b.ih, accR);
    accI = mfma_bf16(a.rl, b.ih, accI);
    accI = mfma_bf16(a.rh, b.il, accI);
    accI = mfma_bf16(a.il, b.rh, accI);
    accI = mfma_bf16(a.ih, b.rl, accI);
    accI = mfma_bf16(a.rh, b.ih, accI);
    accI = mfma_bf16(a.ih, b.rh, accI);
}

template <typename T> __device__ __forceinline__ int acc_row(int lane, int r);
template <> __device__ __forceinline__ int acc_row<double>(int lane, int r) { return (lane >> 4) + 4 * r; }
template <> __device__ __forceinline__ int acc_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }

template <typename T> __device__ __forceinline__ C2<T> cmake(T re, T im) {
    C2<T> v; v.x = re; v.y = im; return v;
}
template <typename T> __device__ __forceinline__ C2<T> czero() { return cmake<T>(T(0), T(0)); }
template <typename T> __device__ __forceinline__ C2<T> cconj(C2<T> a) { return cmake<T>(a.x, -a.y); }
template <typename T> __device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
    return cmake<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) {
    return cmake<T>(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }
template <typename T> __device__ __forceinline__ C2<T> from_d2(double2 v) {
    return cmake<T>(T(v.x), T(v.y));
}

// Device-side per-split result (one truncated SVD).
struct DevInfo {
    int kept;
    int numeric_error;     // non-finite values met
    double discarded;
    double total;
    double entropy;
    unsigned long long offmax_bits;  // max relative off-diagonal of the sweep (bits of a double >= 0)
    int rotations;         // pairs rotated in the sweep
    int inner_steps;       // inner Jacobi steps executed in the sweep (all pairs)
    int scale_exp;         // X is held scaled by 2^scale_exp during the sweeps (FP32 storage)
    int done;              // set on the device once the sweeps converged (1) or hit the limit (2)
    int sweeps;            // sweeps run in this decomposition
    long long rot_total;   // rotated pairs summed over its sweeps
    int qr_fail;           // a Cholesky QR pass met a pivot below its bound (rank deficiency)
    double qr_shift;       // shift of the first Cholesky QR pass
    double gram_trace;     // trace of the Gram matrix of the eigen start's check
    double rest_weight;    // weight of the columns a subset eigen start left out
};

}  // namespace mpo

// ----------------------------------------------------------------- launchers
// Column-major storage everywhere.  op = 0: as stored; op = 1: conjugate transpose.
namespace mpo {
// bf3 selects the split-BF16x3 products (FP32 storage only).
template <typename T>
void launch_cgemm(int opa, int opb, int M, int N, int K, const C2<T>* A, int lda,
                  const C2<T>* B, int ldb, C2<T>* C, int ldc, hipStream_t st, bool bf3 = false);

// X[(a + chiL*I) + ldx*(J + 4c)] = sum M[4I+J][4I'+J'] * theta[(I',a),(J',c)],
// theta = L(As) * R(Bs), ldx >= 4 chiL; also written to X2 (same stride) when non-null.
template <typename T>
void launch_theta_channel(int chiL, int chiM, int chiR, const C2<T>* As, const C2<T>* Bs,
                          const C2<T>* Mdev, C2<T>* X, C2<T>* X2, int ldx, hipStream_t st,
                          bool bf3 = false);

// Eigen-decomposition of the split's Gram matrix (heev.hip): workspace carved
// from the handle's arena, sized for at most cap_m rows and cap_n columns.
constexpr int kTrdNb = 32;            // panel width of the tridiagonalisation
struct HeevFailure { const char* what; };
struct HeevWork {
    double2* Xd;                      // FP64 copy of X, column stride ((cap_m + 1) & ~1) + 8
    double2* G;                       // Gram (stride N + 8), then the reflectors below its diagonal
    double2 *VW, *WV;                 // panel [V W] and [W V], N x 2 kTrdNb each (stride N)
    double2* ypart;                   // slots of the trailing product, (N / 64 + 2) x N (stride N)
    double2 *upart, *tau;             // tiles' parts of u^H G u; reflector scalars
    double* part;                     // partial sums of ||column||^2 (row chunks)
    double2* pdot;                    // partial sums of the panel dots
    double2* pfin;                    // a column's reduced norm and panel dots
    double *d, *e;                    // tridiagonal
    double2 *Sall, *Cpart, *P;        // back-transformation: Y^H Y per block, split-K partials, (X Y) T
    double *Z, *Z2, *U;               // eigenvectors of T and merge scratch (N x N, stride N)
    double *dv, *ds, *dz, *ndv, *ndz, *dfv, *taus, *lam, *zh;
    int *dcol, *ndc, *dfc, *orig, *perm;
    int2* rot_ab;
    double2* rot_cs;
    int *mk, *mnrot;
    double* mrho;
    void* plans;                      // divide-and-conquer plans per size (host, owned by the handle)
    int cap_m = 0, cap_n = 0;
    long long n_runs = 0;
};
size_t heev_bytes(int m_max, int n_max);
void heev_carve(char* p, int m_max, int n_max, HeevWork& w);
void* heev_plans_new();
void heev_plans_free(void* plans);
// X (m x N, stride ld) <- X V with V the eigenvectors of X^H X, computed in FP64;
// with keep < N (and rest non-null) only the keep of the largest eigenvalues,
// X (m x keep), and *rest (device) <- the sum of the other eigenvalues.  Returns
// the number of columns written.
template <typename T>
int heev_precondition(C2<T>* X, int m, int N, int ld, int keep, double* rest, HeevWork& w, Profiler& pf,
                      hipStream_t st);
// A (m x r, stride lda) = Q R: Q (stride ldq, may alias A) an isometry, R (r x r, stride r)
// upper triangular; shifted Cholesky QR plus two Cholesky QR passes in FP64.
// Returns false, writing neither Q nor R, when A is numerically rank-deficient
// (a pivot below its pass's bound); reads that flag through info_host (pinned).
template <typename T>
bool cholqr3(const C2<T>* A, int m, int r, int lda, C2<T>* Q, int ldq, C2<T>* R, DevInfo* info,
             DevInfo* info_host, HeevWork& w, Profiler& pf, hipStream_t st);
// Certificate of the eigen start: true when the largest relative off-diagonal of
// X^H X (FP64, over columns above the floor zrel2) is at most tol.  Synchronises.
template <typename T>
bool heev_check(C2<T>* X, int m, int N, int ld, double tol, double zrel2, DevInfo* info, DevInfo* info_host,
                HeevWork& w, Profiler& pf, hipStream_t st);
// Eigenvalues (ascending) and eigenvectors of a host Hermitian matrix (row-major,
// interleaved complex), through the same kernels.
void heev_host(int N, const double* G, double* w, double* V, HeevWork& work, Profiler& pf, hipStream_t st);

struct JacobiWork {
    void* gram_partials;   // P_max * splits * 64*64 complex (T)
    void* w;               // P_max * 64*64 complex (T)
    int* skip;             // P_max
    double* nrm2;          // N
    int* colmap;           // N (padded)
    double* sig2;          // N, sorted descending
    DevInfo* info;
    DevInfo* info_host;    // pinned
    int max_pairs;
    int splits;
    Profiler* prof;        // may be off
    int block;             // Jacobi block width: 16 or 32 columns
    int inner;             // inner FP64 sweeps per block pair
    bool bf3;              // Gram as split-BF16x3 products (FP32 storage)
    bool trace;            // print each sweep's convergence to stderr
    bool graphs;           // replay captured sweeps (hipGraph) speculatively, one read per batch
    void* graph_cache;     // captured sweep per shape (owned by the handle)
    long long n_splits, n_sweeps, n_rounds, n_rotations;   // running counters
    HeevWork* heev;        // Gram eigen-decomposition start (null = plain sweeps)
    int precond_min;       // start from it for splits with at least this many columns
    long long n_precond;   // splits that started from it
    long long n_checks;    // of those, splits the Gram certificate finished (no sweep)
    int n_cols;            // columns the last decomposition orthogonalised (<= N)
    bool rest_on;          // it left columns out: their weight is info->rest_weight
};

// One-sided block Jacobi on the columns of X (m x N, column stride ld >= m).  On return
// work.colmap[0..n) lists columns by decreasing norm and work.sig2 holds the
// sorted squared norms, n = work.n_cols.  n < N only with keep_max > 0 (the
// caller keeps at most keep_max columns) and the eigen start: then X holds
// the n columns of the largest eigenvalues of X^H X and the
// weight of the others is info->rest_weight (work.rest_on).  Returns the
// number of sweeps, or -1 if the sweep limit was reached, -2 on a HIP error.
template <typename T>
int jacobi_orthogonalize(C2<T>* X, int m, int N, int ld, double tol, int max_sweeps,
                         JacobiWork& w, hipStream_t st, int keep_max = 0);
// Cache of captured sweeps (JacobiWork::graph_cache), created and freed by the handle.
void* jacobi_graph_cache_new();
void jacobi_graph_cache_free(void* cache);

// Columns whose squared norm is at most this fraction of ||X||_F^2 are at the
// rounding floor of the working precision: the sweep never rotates them and
// the truncation never keeps them.  In FP32 storage the rounding of rotated
// columns leaves noise near (2^-24 sqrt(#rotations))^2 ~ 4e-12 of ||X||_F^2;
// both FP32-storage modes use 1e-11, just above it.  (A floor of 1e-9 was 7%
// faster but dropped real Schmidt values of amplitude up to 3e-5 at every
// re-gauge: <Z_i> on an exact 8-qubit circuit moved by 3.7e-5 against 1.1e-5.)
template <typename T> constexpr double jacobi_zero_rel2() { return sizeof(T) == 8 ? 1e-30 : 1e-11; }
constexpr double kZeroRel2Bf3 = jacobi_zero_rel2<float>();   // split-BF16x3 uses the same floor
// Relative orthogonality the FP32-storage sweeps reach with an FP32-MFMA Gram.
// In split-BF16x3 mode the sweeps with the BF16x3 Gram stop at the looser
// tolerance its 16-bit products allow, and sweeps with the FP32-MFMA Gram then
// polish the columns to this one, so that every isometry the mode produces is
// as orthonormal as in FP32 mode.
constexpr double kTolFp32 = 2e-6;
constexpr double kBf3Handoff = 3e-3;

// Truncation + entropy from the sorted squared norms (single work-group); with
// with_rest, info->rest_weight is the weight of further (discarded) values.
void launch_truncate(const double* sig2, int N, int chi_max, double cutoff, double floor_rel2,
                     DevInfo* info, hipStream_t st, bool with_rest = false);

// dst[i + ldd*b] = X[i + ldx*colmap[b]] / sqrt(sig2[b]) for b < k, i < m  (left factor;
// without normalize the columns are copied as they are: U Sigma)
template <typename T>
void launch_gather_cols(const C2<T>* X, int m, int ldx, const int* colmap, const double* sig2, int k,
                        C2<T>* dst, int ldd, hipStream_t st, bool normalize = true);
// dst[b + k*i] = conj(X[i + ldx*colmap[b]]) / sqrt(sig2[b]) for b < k, i < m  (right factor, rows)
template <typename T>
void launch_gather_rows_conj(const C2<T>* X, int m, int ldx, const int* colmap, const double* sig2,
                             int k, C2<T>* dst, hipStream_t st);
// Y[j + ldy*i] = conj(A[i + lda*j])  (A rows x cols with stride lda >= rows, Y cols x rows
// with stride ldy >= cols)
template <typename T>
void launch_conj_transpose(const C2<T>* A, int rows, int cols, int lda, C2<T>* Y, int ldy,
                           hipStream_t st);
// dst[i + ldd*j] = src[i + lds*j] for i < rows, j < cols
template <typename T>
void launch_copy_cols(const C2<T>* src, int rows, int cols, int lds, C2<T>* dst, int ldd, hipStream_t st);
template <typename T>
void launch_copy(const C2<T>* src, C2<T>* dst, size_t count, hipStream_t st);

// Transfer contraction (Sec. III.D): env_out[b] = sum_{a,I} env_in[a] v[I] A[a,I,b]
template <typename T>
void launch_transfer_left(const C2<T>* A, int chiL, int chiR, const double2* env_in,
                          const double2* v, double2* env_out, hipStream_t st);
// env_out[a] = sum_{I,b} A[a,I,b] v[I] env_in[b]; partial: scratch >= chiL*chunks
template <typename T>
void launch_transfer_right(const C2<T>* A, int chiL, int chiR, const double2* env_in,
                           const double2* v, double2* env_out, double2* scratch, hipStream_t st);
// A[a, I, c] *= fl(a) fr(c), fl = lamL[a] or 1/lamL[a] (invL), fr likewise; null = 1
template <typename T>
void launch_scale_site(C2<T>* A, int chiL, int chiR, const double* lamL, const double* lamR, bool invL,
                       bool invR, hipStream_t st);
// A[a, I, b] = [b == a + chiA*I]: the (chiA, 4, 4 chiA) identity site tensor
template <typename T>
void launch_identity_site(C2<T>* A, int chiA, hipStream_t st);
// out[4I+J][4K+L] = sum_{a,c} conj(X[(I,a),(J,c)]) Y[(K,a),(L,c)] (two-site blocks)
template <typename T>
void launch_local_grad(const C2<T>* X, const C2<T>* Y, int chiA, int chiC, double2* out,
                       hipStream_t st);
// Sequential conditional sampling (Sec. III.D): L = 1, logN = 0, clamped = 0 for
// count samples; then per site the marginals of both dits, the draw and the new
// environment (one work-group per sample).
template <typename T>
void launch_sample_init(C2<T>* L, double* logN, int* clamped, int count, hipStream_t st);
template <typename T>
void launch_sample_site(const C2<T>* Ybar, int chiR, int count, const double2* Rk, const double2* v,
                        const double* u, int n, int site, C2<T>* Lnew, unsigned char* bits,
                        double* logN, int* clamped, hipStream_t st);
// out[slot] = sum_a x[a] * y[a]
void launch_dot(const double2* x, const double2* y, int len, double2* out, hipStream_t st);
}  // namespace mpo

// Hermitian eigen-decomposition of a split's Gram matrix, used to hand the
// one-sided Jacobi SVD a starting basis whose columns are already orthogonal
// to about the eigen-solver's accuracy (App. A: the truncated SVD of the
// two-site block; its right singular vectors are the eigenvectors of
// theta'^H theta').  With that basis the Jacobi sweeps only polish: in FP64
// storage one rotating sweep and a check, in FP32 storage a check.
//
//   G = X^H X                  FP64 MFMA
//   G = Q_H T Q_H^H            blocked Householder tridiagonalisation (panels of
//                              kTrdNb columns, rank-2*kTrdNb trailing updates on MFMA)
//   T = Z diag(lambda) Z^T     divide and conquer on the real tridiagonal
//                              (rank-one tearing, secular equation per root,
//                              Gu-Eisenstat vectors, MFMA merge products)
//   X <- X Q_H Z               blocked reflectors (compact WY) + real MFMA GEMM
//
// Everything runs in FP64 whatever the storage precision of X: X is copied to
// FP64 first and the final product is rounded to the storage precision.  The
// columns of the result are then orthogonal relative to their own norms, so
// small singular values are resolved as well as the FP64 Gram allows.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <vector>

#include "common.h"

namespace mpo {

namespace {

constexpr int kPart = 64;          // row chunks of the tridiagonalisation's vector kernels
static_assert(kPart == 64, "the kernels sum the kPart partials one per lane of a wave");
constexpr int kBtNb = 64;          // reflectors per block of the back-transformation
constexpr int kSplitK = 512;       // K chunk of the split-K products

// ------------------------------------------------------------ wave reductions
// Lane l's value to the whole wave (l uniform).
__device__ __forceinline__ double lane_bcast(double v, int l) {
    const unsigned long long x = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x & 0xffffffffull), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The value of the lane that DPP control CTRL pairs with this one.
template <int CTRL>
__device__ __forceinline__ double dpp_pair(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes, the same in every lane, in a fixed order: pairs
// (lane ^ 1), quads (lane ^ 2), then the 8- and 16-lane mirrors within each row
// of 16 on the DPP network, and the four row sums read from lanes 0, 16, 32,
// 48.  Every lane of the wave must be active.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_pair<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_pair<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_pair<0x141>(v);   // row_half_mirror
    v += dpp_pair<0x140>(v);   // row_mirror
    return (lane_bcast(v, 0) + lane_bcast(v, 16)) + (lane_bcast(v, 32) + lane_bcast(v, 48));
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_prod(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v *= __shfl_xor(v, o, 64);
    return v;
}

// Sum of one value per thread over a work-group of NT threads (fixed tree).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) s += red[q];
    __syncthreads();
    return s;
}

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 zcmul(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ double2 zmulc(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// ------------------------------------------------------------ booked launches
// A launch that, with profiling on, carries start/stop events stamped by the
// dispatch itself (hipExtLaunchKernel) and is booked under class cls.
template <typename K, typename... Args>
void launch_booked(Profiler& pf, int cls, double fl, double by, K kernel, dim3 g, dim3 b, size_t lds,
                   hipStream_t st, Args... args) {
    if (pf.on) {
        hipEvent_t a = nullptr, e = nullptr;
        pf.stamps(a, e);
        hipExtLaunchKernelGGL(kernel, g, b, lds, st, a, e, 0, args...);
        pf.record(cls, a, e, fl, by);
    } else {
        hipLaunchKernelGGL(kernel, g, b, lds, st, args...);
    }
}

// ------------------------------------------------------------ complex GEMM
// C = op(A) op(B) (MODE 0) or C -= op(A) op(B) (MODE 1); MODE 2 and 3 are the
// same on the 64x64 tiles on or below the diagonal only, MODE 4 and 5 on those
// on or above it (Hermitian results of which one triangle is used), FP64
// complex, 64x64
// tiles, 4 waves of 2x2 16x16 MFMA tiles.  blockIdx.z selects a batch entry:
// the operands are offset by z times their strides and, with kchunk > 0, the
// entry covers K range [z*kchunk, min(K, (z+1)*kchunk)) (split-K partials).
constexpr int ZBM = 64, ZBN = 64, ZBK = 16;

template <int OPA, int OPB, int MODE>
__global__ __launch_bounds__(256) void k_zgemm(int M, int N, int K, int kchunk, const double2* __restrict__ A,
                                               int lda, size_t sA, const double2* __restrict__ B, int ldb,
                                               size_t sB, double2* __restrict__ C, int ldc, size_t sC) {
    __shared__ double2 As[ZBK][ZBM + 1];
    __shared__ double2 Bs[ZBK][ZBN + 1];
    const int z = blockIdx.z;
    A += sA * z;
    B += sB * z;
    C += sC * z;
    if (kchunk > 0) K = min(kchunk, K - z * kchunk);
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int m0 = blockIdx.x * ZBM, n0 = blockIdx.y * ZBN;
    if ((MODE & 2) && m0 < n0) return;   // Hermitian result: lower tiles only
    if ((MODE & 4) && m0 > n0) return;   // upper tiles only
    d4 accR[2][2], accI[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) { accR[bi][bj][r] = 0.0; accI[bi][bj][r] = 0.0; }
    // the next K tile is loaded into registers while the current one is
    // multiplied from LDS, so the global latency overlaps the MFMA work
    double2 ra[4], rb[4];
    auto load_tiles = [&](int k0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = t + 256 * r;
            int i, k;
            if (OPA == 0) { i = e & 63; k = e >> 6; } else { k = e & 15; i = e >> 4; }
            const int gi = m0 + i, gk = k0 + k;
            double2 v = make_double2(0.0, 0.0);
            if (gi < M && gk < K) {
                v = OPA == 0 ? A[gi + (size_t)gk * lda] : A[gk + (size_t)gi * lda];
                if (OPA == 1) v.y = -v.y;
            }
            ra[r] = v;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = t + 256 * r;
            int j, k;
            if (OPB == 0) { k = e & 15; j = e >> 4; } else { j = e & 63; k = e >> 6; }
            const int gj = n0 + j, gk = k0 + k;
            double2 v = make_double2(0.0, 0.0);
            if (gj < N && gk < K) {
                v = OPB == 0 ? B[gk + (size_t)gj * ldb] : B[gj + (size_t)gk * ldb];
                if (OPB == 1) v.y = -v.y;
            }
            rb[r] = v;
        }
    };
    load_tiles(0);
    for (int k0 = 0; k0 < K; k0 += ZBK) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = t + 256 * r;
            if (OPA == 0) As[e >> 6][e & 63] = ra[r];
            else As[e & 15][e >> 4] = ra[r];
            if (OPB == 0) Bs[e & 15][e >> 4] = rb[r];
            else Bs[e >> 6][e & 63] = rb[r];
        }
        __syncthreads();
        if (k0 + ZBK < K) load_tiles(k0 + ZBK);
#pragma unroll
        for (int kk = 0; kk < ZBK; kk += 4) {
            double2 a[2], b[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                a[q] = As[kk + (lane >> 4)][wm * 32 + q * 16 + (lane & 15)];
                b[q] = Bs[kk + (lane >> 4)][wn * 32 + q * 16 + (lane & 15)];
            }
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    accR[bi][bj] = mfma16(a[bi].x, b[bj].x, accR[bi][bj]);
                    accR[bi][bj] = mfma16(-a[bi].y, b[bj].y, accR[bi][bj]);
                    accI[bi][bj] = mfma16(a[bi].x, b[bj].y, accI[bi][bj]);
                    accI[bi][bj] = mfma16(a[bi].y, b[bj].x, accI[bi][bj]);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = m0 + wm * 32 + bi * 16 + acc_row<double>(lane, r);
                const int j = n0 + wn * 32 + bj * 16 + (lane & 15);
                if (i < M && j < N) {
                    double2* c = C + i + (size_t)j * ldc;
                    if (!(MODE & 1)) *c = make_double2(accR[bi][bj][r], accI[bi][bj][r]);
                    else *c = make_double2(c->x - accR[bi][bj][r], c->y - accI[bi][bj][r]);
                }
            }
}

template <int OPA, int OPB, int MODE>
void zgemm(int M, int N, int K, const double2* A, int lda, const double2* B, int ldb, double2* C, int ldc,
           hipStream_t st, int batches = 1, int kchunk = 0, size_t sA = 0, size_t sB = 0, size_t sC = 0,
           Profiler* pf = nullptr, int cls = 0) {
    if (M <= 0 || N <= 0 || batches <= 0) return;
    dim3 grid((M + ZBM - 1) / ZBM, (N + ZBN - 1) / ZBN, batches);
    if (pf && pf->on) {
        hipEvent_t a = nullptr, e = nullptr;
        pf->stamps(a, e);
        hipExtLaunchKernelGGL((k_zgemm<OPA, OPB, MODE>), grid, dim3(256), 0, st, a, e, 0, M, N, K, kchunk, A, lda,
                              sA, B, ldb, sB, C, ldc, sC);
        const double kk = kchunk > 0 ? (double)K : (double)K * batches;
        const double part = (MODE & 6) ? 0.5 : 1.0;   // one triangle's tiles only
        pf->record(cls, a, e, part * 8.0 * M * N * kk,
                   16.0 * ((double)M * kk + (double)N * kk + part * ((MODE & 1) + 1.0) * M * N * batches));
    } else {
        hipLaunchKernelGGL((k_zgemm<OPA, OPB, MODE>), grid, dim3(256), 0, st, M, N, K, kchunk, A, lda, sA, B, ldb,
                           sB, C, ldc, sC);
    }
}

// ------------------------------------------------------------ real GEMM
// One 64x64 tile of C = A B, FP64, A's columns optionally through a map
// (absolute column indices), output converted to TO.
template <typename TO>
__device__ __forceinline__ TO to_out(double v) { return (TO)v; }

template <typename TO, bool MAP>
__device__ __forceinline__ void dgemm_tile(int M, int N, int K, const double* __restrict__ A, int lda,
                                           const int* __restrict__ amap, const double* __restrict__ B, int ldb,
                                           TO* __restrict__ C, int ldc, int m0, int n0) {
    __shared__ double As[ZBK][ZBM + 1];
    __shared__ double Bs[ZBK][ZBN + 1];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    d4 acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[bi][bj][r] = 0.0;
    for (int k0 = 0; k0 < K; k0 += ZBK) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = t + 256 * r;
            const int i = e & 63, k = e >> 6;
            const int gi = m0 + i, gk = k0 + k;
            double v = 0.0;
            if (gi < M && gk < K) v = A[gi + (size_t)(MAP ? amap[gk] : gk) * lda];
            As[k][i] = v;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = t + 256 * r;
            const int k = e & 15, j = e >> 4;
            const int gj = n0 + j, gk = k0 + k;
            Bs[k][j] = (gj < N && gk < K) ? B[gk + (size_t)gj * ldb] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < ZBK; kk += 4) {
            double a[2], b[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                a[q] = As[kk + (lane >> 4)][wm * 32 + q * 16 + (lane & 15)];
                b[q] = Bs[kk + (lane >> 4)][wn * 32 + q * 16 + (lane & 15)];
            }
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = mfma16(a[bi], b[bj], acc[bi][bj]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = m0 + wm * 32 + bi * 16 + acc_row<double>(lane, r);
                const int j = n0 + wn * 32 + bj * 16 + (lane & 15);
                if (i < M && j < N) C[i + (size_t)j * ldc] = to_out<TO>(acc[bi][bj][r]);
            }
}

template <typename TO>
__global__ __launch_bounds__(256) void k_dgemm(int M, int N, int K, const double* __restrict__ A, int lda,
                                               const double* __restrict__ B, int ldb, TO* __restrict__ C,
                                               int ldc) {
    dgemm_tile<TO, false>(M, N, K, A, lda, nullptr, B, ldb, C, ldc, blockIdx.x * ZBM, blockIdx.y * ZBN);
}

// ------------------------------------------------------------ Gram, copies
template <typename T>
__global__ __launch_bounds__(256) void k_to_f64(const C2<T>* __restrict__ X, int m, int ld, double2* __restrict__ Xd,
                                                int ldd) {
    const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
    if (i < m) Xd[i + (size_t)ldd * j] = to_d2(X[i + (size_t)ld * j]);
}

__global__ void k_fill_z(double2* p, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = make_double2(0.0, 0.0);
}

// ------------------------------------------- Householder tridiagonalisation
// Lower storage of the Hermitian G (both triangles kept valid by the trailing
// updates).  Reflector j: H_j = I - tau_j v v^H with v[0..j] = 0, v[j+1] = 1,
// beta_j = -sign(Re alpha) ||G[j+1:, j]|| real, so that T is real symmetric
// with diagonal d and off-diagonal e.  Within a panel (columns j0..j0+nb-1)
// the trailing matrix is left as it was at the panel start and corrected on
// the fly by the panel's V and W (G_eff = G - V W^H - W V^H); after the panel
// it is updated once by a rank-2 nb product on MFMA.

struct House { double2 tau, scale; double beta; };

// Reflector scalars of column j from alpha = G[j+1, j] and ||G[j+2:, j]||^2.
__device__ __forceinline__ House house_scalars(double2 alpha, double xnorm2) {
    House h;
    if (xnorm2 == 0.0 && alpha.y == 0.0) {
        h.tau = make_double2(0.0, 0.0);
        h.scale = make_double2(0.0, 0.0);
        h.beta = alpha.x;
        return h;
    }
    const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xnorm2);
    const double beta = alpha.x >= 0.0 ? -nrm : nrm;
    h.beta = beta;
    h.tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
    const double2 den = make_double2(alpha.x - beta, alpha.y);   // |den| >= |beta|: no cancellation
    const double dd = den.x * den.x + den.y * den.y;
    h.scale = make_double2(den.x / dd, -den.y / dd);
    return h;
}

// Row chunk of kPart work-groups over [r0, N).
__device__ __forceinline__ void part_rows(int r0, int N, int& a, int& b) {
    const int len = N - r0;
    const int ch = len > 0 ? (len + kPart - 1) / kPart : 0;
    a = r0 + (int)blockIdx.x * ch;
    b = min(N, a + ch);
}

// Panel start: partial sums of ||G[j+2:, j]||^2 (column j needs no panel update).
__global__ __launch_bounds__(256) void k_trd_colnorm(const double2* __restrict__ G, int ldg, int N, int j,
                                                     double* __restrict__ part) {
    __shared__ double red[4];
    int a, b;
    part_rows(j + 2, N, a, b);
    double s = 0.0;
    for (int i = a + (int)threadIdx.x; i < b; i += 256) {
        const double2 v = G[i + (size_t)ldg * j];
        s += v.x * v.x + v.y * v.y;
    }
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Column j of the panel (c = j - j0).  With G0 the panel-start trailing matrix
// G[j+1:, j+1:] (as stored: the panel's updates are deferred) and the
// reflector v = e_0 + scale u, u = [0, x], x = G[j+2:, j] as stored,
//   G_eff v = G0 e_0 + scale G0 u - V (W^H v) - W (V^H v):
// G0 e_0 is the stored column G[j+1:, j+1], and the tile product G0 u needs
// neither the reflector's scalars nor the panel.  k_trd_hemv forms G0 u from
// the lower triangle only, in 64x64 tiles, one work-group per tile (I, J),
// I >= J (tile coordinates from the trailing origin j+1):
//   tile I > J     row partials G_IJ u_J (rows of block I) and column partials
//                  G_IJ^H u_I (rows of block J), each into its own slot of
//                  ypart: block K's rows collect slot J from tile (K, J), slot
//                  I from tile (I, K), and slots K and nt from the diagonal
//                  tile (its strict lower part both ways, the real diagonal
//                  once), nt + 1 slots in all, summed by k_trd_step;
//   per tile       its part of u^H G0 u (u_I^H G_IJ u_J + u_J^H G_IJ^H u_I,
//                  the diagonal tile's lower part with its real diagonal) in
//                  upart[tile].
constexpr int kHt = 64;   // tile edge of the trailing product

// Tile t of the lower triangle of an nt x nt tile grid, numbered down the
// tile columns (J = 0: I = 0 .. nt-1, then J = 1: I = 1 .. nt-1, ..), so that
// work-groups with neighbouring numbers read neighbouring kilobytes of each
// column of G.
__device__ __forceinline__ void lower_tile(int t, int nt, int& I, int& J) {
    // columns before J hold J nt - J (J - 1) / 2 tiles
    const double b = 2.0 * nt + 1.0;
    int jj = (int)((b - sqrt(b * b - 8.0 * t)) * 0.5);
    jj = max(0, min(jj, nt - 1));
    while (jj > 0 && jj * nt - jj * (jj - 1) / 2 > t) --jj;
    while (jj + 1 < nt && (jj + 1) * nt - (jj + 1) * jj / 2 <= t) ++jj;
    J = jj;
    I = jj + (t - (jj * nt - jj * (jj - 1) / 2));
}

__global__ __launch_bounds__(256) void k_trd_hemv(const double2* __restrict__ G, int ldg, int N, int j,
                                                  double2* __restrict__ ypart, double2* __restrict__ upart, int c,
                                                  const double* __restrict__ part, const double2* __restrict__ pdot,
                                                  double2* __restrict__ pfin) {
    __shared__ double2 uI[kHt], uJ[kHt];
    __shared__ double2 red[16][kHt];
    __shared__ double2 ured[4];
    const int len = N - j - 1;
    const int nt = (len + kHt - 1) / kHt;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if ((int)blockIdx.x == nt * (nt + 1) / 2) {
        // the last work-group: the column's sums for k_trd_step from the row
        // chunks' partials, ||G[j+2:, j]||^2 into pfin[0].x and the panel dots
        // (W^H x)_q, (V^H x)_q into pfin[1 + q], pfin[1 + kTrdNb + q], q < c;
        // thread (dot dd, sub) adds partials sub, sub + 8, .., then the eight
        // subs are summed on the DPP network
        if (wave == 0) {
            const double sn = wave_sum(part[lane]);
            if (lane == 0) pfin[0] = make_double2(sn, 0.0);
        }
        const int dsub = tid & 7;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int dd = (tid >> 3) + 32 * hh;          // pfin index - 1: p_q (dd < kTrdNb), q_q
            const bool live = (dd % kTrdNb) < c;
            double2 sd = make_double2(0.0, 0.0);
            if (live) {
#pragma unroll
                for (int k = 0; k < kPart / 8; ++k) {
                    const double2 v = pdot[(size_t)(dsub + 8 * k) * 2 * kTrdNb + dd];
                    sd.x += v.x;
                    sd.y += v.y;
                }
            }
            sd.x += dpp_pair<0xB1>(sd.x);
            sd.y += dpp_pair<0xB1>(sd.y);
            sd.x += dpp_pair<0x4E>(sd.x);
            sd.y += dpp_pair<0x4E>(sd.y);
            sd.x += dpp_pair<0x141>(sd.x);
            sd.y += dpp_pair<0x141>(sd.y);
            if (live && dsub == 0) pfin[1 + dd] = sd;
        }
        return;
    }
    int I, J;
    lower_tile((int)blockIdx.x, nt, I, J);
    // lane (p, q) = (lane % 8, lane / 8) takes rows 8 s + p and columns
    // 16 wave + 8 cc + q, so each load instruction reads eight 128-byte row runs
    const int p = lane & 7, q = lane >> 3;
    const int rows = min(kHt, len - kHt * I), cols = min(kHt, len - kHt * J);
    const double2* T0 = G + (size_t)(j + 1 + kHt * I) + (size_t)ldg * (j + 1 + kHt * J);
    double2 a[8][2];
#pragma unroll
    for (int s8 = 0; s8 < 8; ++s8)
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            const int r = 8 * s8 + p, b = 16 * wave + 8 * cc + q;
            const bool ok = r < rows && b < cols && (I != J || r >= b);
            a[s8][cc] = ok ? T0[r + (size_t)ldg * b] : make_double2(0.0, 0.0);
        }
    // u = [0, G[j+2:, j]] on the tile's row and column blocks
    const double2* colj = G + (size_t)ldg * j + (j + 1);
    if (tid < 128) {
        const int r = kHt * (tid < 64 ? I : J) + (tid & 63);
        double2 u = make_double2(0.0, 0.0);
        if (r > 0 && r < len) u = colj[r];
        if (tid < 64) uI[tid] = u;
        else uJ[tid - 64] = u;
    }
    __syncthreads();
    double2 racc[8], cacc[2];
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) cacc[cc] = make_double2(0.0, 0.0);
#pragma unroll
    for (int s8 = 0; s8 < 8; ++s8) {
        racc[s8] = make_double2(0.0, 0.0);
        const int r = 8 * s8 + p;
        const double2 ui = uI[r];
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            const int b = 16 * wave + 8 * cc + q;
            double2 g = a[s8][cc];
            const bool diag = I == J && r == b;
            if (diag) g.y = 0.0;                   // Hermitian: real diagonal, counted once
            const double2 ub = uJ[b];
            racc[s8].x += g.x * ub.x - g.y * ub.y;
            racc[s8].y += g.x * ub.y + g.y * ub.x;
            if (!diag) {                            // conj(g) u_r into y_b
                cacc[cc].x += g.x * ui.x + g.y * ui.y;
                cacc[cc].y += g.x * ui.y - g.y * ui.x;
            }
        }
    }
    // rows: sum over q (lane bits 3..5): lane ^ 8 on the DPP network (row_ror:8
    // within each row of 16 lanes), then the four rows of 16 and the four waves
    // through LDS; columns: sum over p (lane bits 0..2) on the DPP network
#pragma unroll
    for (int s8 = 0; s8 < 8; ++s8) {
        racc[s8].x += dpp_pair<0x128>(racc[s8].x);
        racc[s8].y += dpp_pair<0x128>(racc[s8].y);
    }
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
        cacc[cc].x += dpp_pair<0xB1>(cacc[cc].x);
        cacc[cc].y += dpp_pair<0xB1>(cacc[cc].y);
        cacc[cc].x += dpp_pair<0x4E>(cacc[cc].x);
        cacc[cc].y += dpp_pair<0x4E>(cacc[cc].y);
        cacc[cc].x += dpp_pair<0x141>(cacc[cc].x);
        cacc[cc].y += dpp_pair<0x141>(cacc[cc].y);
    }
    const size_t ldy = (size_t)N;
    double2 uu = make_double2(0.0, 0.0);   // this lane's part of u^H G0 u
    if ((q & 1) == 0) {
#pragma unroll
        for (int s8 = 0; s8 < 8; ++s8) {
            red[4 * wave + (q >> 1)][8 * s8 + p] = racc[s8];
            const double2 t = zcmul(uI[8 * s8 + p], racc[s8]);
            uu.x += t.x;
            uu.y += t.y;
        }
    }
    if (p == 0) {
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            const double2 t = zcmul(uJ[16 * wave + 8 * cc + q], cacc[cc]);
            uu.x += t.x;
            uu.y += t.y;
        }
    }
    uu.x = wave_sum(uu.x);
    uu.y = wave_sum(uu.y);
    if (lane == 0) ured[wave] = uu;
    if (p == 0) {
        const int slot = I == J ? nt : I;
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            const int b = 16 * wave + 8 * cc + q;
            if (b < cols) ypart[(size_t)slot * ldy + kHt * J + b] = cacc[cc];
        }
    }
    __syncthreads();
    if (tid < rows) {
        double2 sr = red[0][tid];
#pragma unroll
        for (int w4 = 1; w4 < 16; ++w4) { sr.x += red[w4][tid].x; sr.y += red[w4][tid].y; }
        ypart[(size_t)J * ldy + kHt * I + tid] = sr;
    }
    if (tid == 0) {
        double2 su = ured[0];
        for (int w4 = 1; w4 < 4; ++w4) { su.x += ured[w4].x; su.y += ured[w4].y; }
        upart[blockIdx.x] = su;
    }
}

// The rest of column j in one kernel over kPart row chunks of all N rows, every
// work-group forming the column's scalars itself (the same sums in the same
// order in each):
//   reflector      tau_j, scale s, beta from alpha = G[j+1, j] and
//                  ||G[j+2:, j]||^2; v = e_0 + s u;
//   panel dots     p = W^H v, q = V^H v from W^H x and V^H x;
// (the two sums come reduced from the last work-group of k_trd_hemv, which
// adds up the partials the previous column's kernel left);
//   y              y_i = G[i, j+1] + s (G0 u)_i - (V p + W q)_i, (G0 u)_i the
//                  sum of row i's slots of the tile product;
//   alpha          = -|tau|^2 (v^H G_eff v) / 2 (real, G_eff Hermitian) with
//                  v^H G_eff v = G0[0, 0] + 2 Re(s (G0 u)_0) + |s|^2 u^H G0 u
//                  - 2 Re(q^H p), u^H G0 u from the tiles' partial sums;
//   panel column   w = tau y + alpha v into the panel buffers (zero above row
//                  j+1), v into them and below the diagonal of G (G[j+1, j] =
//                  1 for the back-transformation);
// and, if the panel continues, column j+1 brought up to date,
// G[j+1:, j+1] -= V conj(W[j+1, :]) + W conj(V[j+1, :]) over the panel's
// first c+1 columns, with the partial sums its reflector needs:
// ||G[j+3:, j+1]||^2, W^H G[j+3:, j+1] and V^H G[j+3:, j+1].
// Every global load is issued at the start (the chunk's panel rows go to LDS),
// so the kernel waits on memory once; the rest is LDS work between barriers.
// Nothing another work-group of the same launch reads is written: the partial
// sums for column j+1 go to the other half of double-buffered arrays, G[j+1, j]
// and G[j+1, j+1] are left as they are (d[j+1] takes the updated diagonal).
constexpr int kStepG = 8;                                  // row groups (waves) of k_trd_step
constexpr int kStepSlots = (64 * kPart / kHt + 1 + kStepG - 1) / kStepG;   // slots per thread (nt + 1 <= 65)
constexpr int kUpartPer = 5;   // tile partials per thread: 512 * 5 >= 64 * 65 / 2

__global__ __launch_bounds__(64 * kStepG) void k_trd_step(double2* __restrict__ G, int ldg, int N, int j, int c,
                                                  int update_next, const double2* __restrict__ ypart,
                                                  const double2* __restrict__ upart, double2* __restrict__ VW,
                                                  double2* __restrict__ WV, const double2* __restrict__ pfin,
                                                  double* __restrict__ part_next,
                                                  double2* __restrict__ pdot_next, double2* __restrict__ tau,
                                                  double* __restrict__ d, double* __restrict__ e) {
    __shared__ double2 Vc[kTrdNb][65];    // V[a + r, q] as Vc[q][r] (q < c)
    __shared__ double2 Wc[kTrdNb][65];
    __shared__ double2 red4[kStepG][64];
    __shared__ double2 row1[2 * kTrdNb];  // V[j+1, q], W[j+1, q] for q < c
    __shared__ double2 pq[2 * kTrdNb];    // p, then q
    __shared__ double2 sv[64], sw[64];    // v and w on this chunk's rows
    __shared__ double2 arow[64];          // updated column j+1 on this chunk's rows (>= j+3; else 0)
    __shared__ double ured[kStepG];
    __shared__ double2 sy0;               // (G0 u)_0
    const double2 zero = make_double2(0.0, 0.0);
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int len = N - j - 1;
    const int nt = (len + kHt - 1) / kHt;
    const int ntiles = nt * (nt + 1) / 2;
    int a, b;
    part_rows(0, N, a, b);
    const int nr = b - a;                 // <= 64
    const int r = t & 63, g = t >> 6;     // (row, group)
    const int i = a + r;
    const bool trow = r < nr && i > j;    // a trailing row
    const int tr = i - j - 1;             // its index in the trailing part
    const size_t ldy = (size_t)N;
    // ---- global loads
    double2 sl[kStepSlots];
#pragma unroll
    for (int k = 0; k < kStepSlots; ++k) {
        const int s = g + kStepG * k;
        sl[k] = zero;
        if (trow && s <= nt) sl[k] = ypart[(size_t)s * ldy + tr];
    }
    // panel rows of the chunk, columns q = g + kStepG k < c (a condition that is
    // the same for the whole wave)
    double2 pv[kTrdNb / kStepG], pw[kTrdNb / kStepG];
    const int ic = min(i, N - 1);
#pragma unroll
    for (int k = 0; k < kTrdNb / kStepG; ++k) {
        const int q = g + kStepG * k;
        pv[k] = zero;
        pw[k] = zero;
        if (q < c) {
            pv[k] = VW[ic + (size_t)N * q];
            pw[k] = VW[ic + (size_t)N * (kTrdNb + q)];
        }
    }
    double upv[kUpartPer];
#pragma unroll
    for (int k = 0; k < kUpartPer; ++k) upv[k] = upart[min(t + 64 * kStepG * k, ntiles - 1)].x;
    double2 g0 = zero, xi = zero;          // G[i, j+1] (panel start), G[i, j]
    if (trow && g == 0) {
        g0 = G[i + (size_t)ldg * (j + 1)];
        xi = G[i + (size_t)ldg * j];
    }
    double2 y0s = zero;
    if (wave == 0) {
        if (lane <= nt) y0s = ypart[(size_t)lane * ldy];
        if (lane == 0 && nt == 64) { const double2 v = ypart[(size_t)64 * ldy]; y0s.x += v.x; y0s.y += v.y; }
    }
    // row j+1 of the panel (r1: V then W, the layout of row1), the entry of it
    // that pq[t] needs (rw: W[j+1, q] for p_q, V[j+1, q] for q_q), and the
    // column's reduced sums from the trailing product's last work-group
    double2 r1 = zero, rw = zero, fd = zero;
    const bool pqt = t < 2 * kTrdNb && (t % kTrdNb) < c;
    if (pqt) {
        r1 = VW[(j + 1) + (size_t)N * t];
        rw = VW[(j + 1) + (size_t)N * ((t < kTrdNb ? kTrdNb : 0) + t % kTrdNb)];
        fd = pfin[1 + t];
    }
    const double xnorm2 = pfin[0].x;
    const double2 alpha = G[(j + 1) + (size_t)ldg * j];
    const double g00 = G[(j + 1) + (size_t)ldg * (j + 1)].x;
    // ---- reflector scalars, panel dots, (G0 u)_0 and u^H G0 u
#pragma unroll
    for (int k = 0; k < kTrdNb / kStepG; ++k) {
        const int q = g + kStepG * k;
        if (q < c) {
            double2 v = pv[k], w = pw[k];
            if (r >= nr) { v = make_double2(0.0, 0.0); w = v; }
            Vc[q][r] = v;
            Wc[q][r] = w;
        }
    }
    double up = 0.0;
#pragma unroll
    for (int k = 0; k < kUpartPer; ++k)
        if (t + 64 * kStepG * k < ntiles) up += upv[k];
    const House h = house_scalars(alpha, xnorm2);
    if (t < 2 * kTrdNb) row1[t] = r1;
    if (pqt) {
        // p_q = conj(W[j+1, q]) + s (W^H x)_q, q_q = conj(V[j+1, q]) + s (V^H x)_q
        const double2 sc = zmul(h.scale, fd);
        pq[t] = make_double2(rw.x + sc.x, -rw.y + sc.y);
    }
    if (wave == 0) {
        const double2 y0 = make_double2(wave_sum(y0s.x), wave_sum(y0s.y));
        if (lane == 0) sy0 = y0;
    }
    up = wave_sum(up);
    if (lane == 0) ured[wave] = up;
    __syncthreads();
    // ---- column scalars (every thread alike)
    double uGu = ured[0];
#pragma unroll
    for (int w8 = 1; w8 < kStepG; ++w8) uGu += ured[w8];
    // the panel's correction to y_{j+1} and Re(q^H p): lane qq < c of every wave
    // takes panel column qq, the wave sums
    double c1r = 0.0, c1i = 0.0, qp = 0.0;
    if (lane < c) {
        const double2 t1 = zmul(row1[lane], pq[lane]);
        const double2 t2 = zmul(row1[kTrdNb + lane], pq[kTrdNb + lane]);
        c1r = t1.x + t2.x;
        c1i = t1.y + t2.y;
        qp = pq[kTrdNb + lane].x * pq[lane].x + pq[kTrdNb + lane].y * pq[lane].y;   // Re(conj(q) p)
    }
    const double corr1r = wave_sum(c1r), corr1i = wave_sum(c1i), qpr = wave_sum(qp);
    const double2 y0 = sy0;
    const double2 sy = zmul(h.scale, y0);
    const double s2 = h.scale.x * h.scale.x + h.scale.y * h.scale.y;
    const double vgv = g00 + 2.0 * sy.x + s2 * uGu - 2.0 * qpr;
    const double t2n = h.tau.x * h.tau.x + h.tau.y * h.tau.y;
    const double al = -0.5 * t2n * vgv;
    const double2 y1 = make_double2(g00 + sy.x - corr1r, sy.y - corr1i);   // y_{j+1}
    const double2 w1t = zmul(h.tau, y1);
    const double2 wj1 = make_double2(w1t.x + al, w1t.y);                     // W[j+1, c] (v_{j+1} = 1)
    // ---- this thread's share of y_i: s (its slots) - (its panel columns of V p + W q)
    {
        double2 acc = zero;
#pragma unroll
        for (int k = 0; k < kStepSlots; ++k) { acc.x += sl[k].x; acc.y += sl[k].y; }
        acc = zmul(h.scale, acc);
#pragma unroll
        for (int k = 0; k < kTrdNb / kStepG; ++k) {
            const int qq = g + kStepG * k;
            if (qq < c) {
                const double2 t1 = zmul(Vc[qq][r], pq[qq]);
                const double2 t2 = zmul(Wc[qq][r], pq[kTrdNb + qq]);
                acc.x -= t1.x + t2.x;
                acc.y -= t1.y + t2.y;
            }
        }
        red4[g][r] = acc;
    }
    __syncthreads();
    if (t < 64) {
        double2 v = zero, w = zero;
        if (trow) {
            if (tr == 0) {
                v = make_double2(1.0, 0.0);
                w = wj1;
            } else {
                double sr = g0.x, si = g0.y;
#pragma unroll
                for (int w8 = 0; w8 < kStepG; ++w8) { sr += red4[w8][t].x; si += red4[w8][t].y; }
                v = zmul(xi, h.scale);
                const double2 wt = zmul(h.tau, make_double2(sr, si));
                w = make_double2(wt.x + al * v.x, wt.y + al * v.y);
            }
            // G[j+1, j] keeps alpha, which every work-group reads; the
            // back-transformation's mask stores the reflector's 1 there
            if (tr > 0) G[i + (size_t)ldg * j] = v;
        }
        if (r < nr) {
            VW[i + (size_t)N * c] = v;
            WV[i + (size_t)N * (kTrdNb + c)] = v;
            VW[i + (size_t)N * (kTrdNb + c)] = w;
            WV[i + (size_t)N * c] = w;
        }
        sv[t] = v;
        sw[t] = w;
        if (blockIdx.x == 0 && t == 0) {
            tau[j] = h.tau;
            e[j] = h.beta;
            if (c == 0) d[j] = G[j + (size_t)ldg * j].x;   // else set by the previous column's update
        }
    }
    if (!update_next) return;
    __syncthreads();
    // column j+1 update: thread (row r, group g) sums the panel columns q = g, g+4, ..
    double2 acc = zero;
    const bool urow = r < nr && i >= j + 1;
    if (urow) {
#pragma unroll
        for (int k = 0; k <= kTrdNb / kStepG; ++k) {   // q = g + kStepG k <= c <= 31
            const int q = g + kStepG * k;
            if (q < c) {
                const double2 t1 = zmulc(Vc[q][r], row1[kTrdNb + q]), t2 = zmulc(Wc[q][r], row1[q]);
                acc.x += t1.x + t2.x;
                acc.y += t1.y + t2.y;
            } else if (q == c) {
                const double2 t1 = zmulc(sv[r], wj1), t2 = sw[r];
                acc.x += t1.x + t2.x;
                acc.y += t1.y + t2.y;
            }
        }
    }
    red4[g][r] = acc;
    __syncthreads();
    if (t < 64) {
        double nrm = 0.0;
        double2 gv = zero;
        if (urow) {
            gv = g0;
            for (int q8 = 0; q8 < kStepG; ++q8) { gv.x -= red4[q8][t].x; gv.y -= red4[q8][t].y; }
            // G[j+1, j+1] keeps its panel-start value, which every work-group
            // reads; its update is the next diagonal entry of T
            if (i == j + 1) d[j + 1] = gv.x;
            else G[i + (size_t)ldg * (j + 1)] = gv;
            if (i >= j + 3) nrm = gv.x * gv.x + gv.y * gv.y;
        }
        double2 av = zero;
        if (urow && i >= j + 3) av = gv;
        arow[t] = av;
        nrm = wave_sum(nrm);
        if (t == 0) part_next[blockIdx.x] = nrm;
    }
    __syncthreads();
    // dots over this chunk: thread (dot r, row group g) sums conj(W[i, q]) a_i
    // (r < c+1) or conj(V[i, q]) a_i (r >= c+1) over rows a + g, a + g + kStepG, ..
    const int nq = c + 1;
    double2 dacc = zero;
    if (r < 2 * nq) {
        const int q = r % nq, isv = r / nq;
#pragma unroll
        for (int k = 0; k < 64 / kStepG; ++k) {
            const int rr = g + kStepG * k;
            if (rr < nr) {
                double2 cval;
                if (q == c) cval = isv ? sv[rr] : sw[rr];
                else cval = isv ? Vc[q][rr] : Wc[q][rr];
                const double2 p = zcmul(cval, arow[rr]);
                dacc.x += p.x;
                dacc.y += p.y;
            }
        }
    }
    red4[g][r] = dacc;
    __syncthreads();
    if (t < 2 * nq) {
        const int q = t % nq, isv = t / nq;
        double2 sum = zero;
        for (int q8 = 0; q8 < kStepG; ++q8) { sum.x += red4[q8][t].x; sum.y += red4[q8][t].y; }
        pdot_next[(size_t)blockIdx.x * 2 * kTrdNb + isv * kTrdNb + q] = sum;
    }
}

__global__ void k_trd_last(const double2* __restrict__ G, int ldg, int N, double* __restrict__ d) {
    if (threadIdx.x == 0 && blockIdx.x == 0) d[N - 1] = G[(N - 1) + (size_t)ldg * (N - 1)].x;
}

// ----------------------------------------------------- divide and conquer
// T = diag(T1', T2') + |beta| u u^T, u = [e_last; sign(beta) e_first] at every
// internal node of a halving tree with leaves of size 1 (the diagonal entries
// on both sides of every coupling lose |beta|).  A merge with children
// T1' = Q1 D1 Q1^T, T2' = Q2 D2 Q2^T solves D + rho z z^T, z = [Q1^T e_last;
// sign(beta) Q2^T e_first] / sqrt(2), rho = 2|beta|:
//   deflation   rho |z_i| <= tol: (d_i, e_i) is an eigenpair; two close values
//               are rotated so that one z component vanishes (tol = 8 eps
//               max(|d|, rho));
//   roots       one per interval (delta_j, delta_{j+1}) (the last in
//               (delta_{k-1}, delta_{k-1} + rho |z|^2]), found by bisection in
//               the coordinate of the nearer pole, so that delta_i - lambda_j
//               keeps full relative accuracy;
//   vectors     z recomputed from the roots (Gu-Eisenstat), u_j = zhat /
//               (delta - lambda_j) normalised: orthogonal to working accuracy;
//   product     [Q1 0; 0 Q2] (rotated, deflated columns removed) times U on MFMA.
// Eigenvalues are kept in ascending order within every node.

__global__ void k_dc_init(int N, const double* __restrict__ d, const double* __restrict__ e,
                          double* __restrict__ dv, double* __restrict__ Z) {
    const size_t nn = (size_t)N * N;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < nn; q += stride) {
        const size_t i = q % N, k = q / N;
        Z[q] = i == k ? 1.0 : 0.0;
        if (k == 0) {
            double v = d[i];
            if (i >= 1) v -= fabs(e[i - 1]);
            if (i + 1 < (size_t)N) v -= fabs(e[i]);
            dv[i] = v;
        }
    }
}

struct DcMerge { int lo, n1, n2, id; };

// number of entries of sorted a[0..n) below x (strict) / at most x
__device__ __forceinline__ int count_less(const double* a, int n, double x) {
    int lo = 0, hi = n;
    while (lo < hi) { const int mid = (lo + hi) >> 1; if (a[mid] < x) lo = mid + 1; else hi = mid; }
    return lo;
}
__device__ __forceinline__ int count_le(const double* a, int n, double x) {
    int lo = 0, hi = n;
    while (lo < hi) { const int mid = (lo + hi) >> 1; if (a[mid] <= x) lo = mid + 1; else hi = mid; }
    return lo;
}

struct DcBuf {
    double *dv, *ds, *dz, *ndv, *ndz, *dfv, *taus, *lam, *zh;
    int *dcol, *ndc, *dfc, *orig, *perm;
    int2* rot_ab;
    double2* rot_cs;
    int *mk, *mnrot;
    double* mrho;
};

// One work-group per merge: z, the merged ascending order, and the deflation
// scan (sequential, thread 0).
__global__ __launch_bounds__(1024) void k_dc_prep(const DcMerge* __restrict__ plan, int N,
                                                  const double* __restrict__ e, const double* __restrict__ Z,
                                                  DcBuf b) {
    const DcMerge mg = plan[blockIdx.x];
    const int lo = mg.lo, n1 = mg.n1, n2 = mg.n2, n = n1 + n2;
    const double beta = e[lo + n1 - 1];
    const double rho = 2.0 * fabs(beta);
    const double sg = beta < 0.0 ? -1.0 : 1.0;
    const double r2 = 0.70710678118654752440;
    const double* dl = b.dv + lo;
    const double* dr = b.dv + lo + n1;
    __shared__ double sds[4096], sdz[4096];
    __shared__ int sdc[4096];
    for (int t = threadIdx.x; t < n; t += 1024) {
        double val, zt;
        int pos;
        if (t < n1) {
            val = dl[t];
            pos = t + count_less(dr, n2, val);
            zt = Z[(lo + n1 - 1) + (size_t)N * (lo + t)] * r2;
        } else {
            const int u = t - n1;
            val = dr[u];
            pos = u + count_le(dl, n1, val);
            zt = sg * Z[(lo + n1) + (size_t)N * (lo + t)] * r2;
        }
        sds[pos] = val;
        sdz[pos] = zt;
        sdc[pos] = lo + t;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    // the scan reads the merged order from LDS and keeps the last kept pole in
    // registers; its results go to global memory with stores it never reads back
    const double dmax = fmax(fabs(sds[0]), fabs(sds[n - 1]));
    const double tol = 8.0 * 2.220446049250313e-16 * fmax(dmax, rho);
    int k = 0, nd = 0, nrot = 0;
    double dlast = 0.0, zlast = 0.0;
    int clast = 0;
    for (int t = 0; t < n; ++t) {
        double dt = sds[t], zt = sdz[t];
        const int ct = sdc[t];
        if (rho * fabs(zt) <= tol) {
            b.dfv[lo + nd] = dt;
            b.dfc[lo + nd] = ct;
            ++nd;
            continue;
        }
        if (k > 0) {
            const double tt = hypot(zlast, zt);
            const double cc = zt / tt, ss = -zlast / tt;
            if (fabs((dt - dlast) * cc * ss) <= tol) {
                b.rot_ab[lo + nrot] = make_int2(clast, ct);
                b.rot_cs[lo + nrot] = make_double2(cc, ss);
                ++nrot;
                const double dnl = dlast * cc * cc + dt * ss * ss;
                const double dnt = dlast * ss * ss + dt * cc * cc;
                --k;
                b.dfv[lo + nd] = dnl;
                b.dfc[lo + nd] = clast;
                ++nd;
                dt = dnt;
                zt = tt;
            }
        }
        b.ndv[lo + k] = dt;
        b.ndz[lo + k] = zt;
        b.ndc[lo + k] = ct;
        dlast = dt;
        zlast = zt;
        clast = ct;
        ++k;
    }
    b.mk[mg.id] = k;
    b.mnrot[mg.id] = nrot;
    b.mrho[mg.id] = rho;
}

// The deflation rotations on the merge's block rows, in scan order.
__global__ __launch_bounds__(256) void k_dc_rot(const DcMerge* __restrict__ plan, int N, double* __restrict__ Z,
                                                DcBuf b) {
    const DcMerge mg = plan[blockIdx.y];
    const int n = mg.n1 + mg.n2, nrot = b.mnrot[mg.id];
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= n || nrot == 0) return;
    const size_t row = mg.lo + r;
    for (int q = 0; q < nrot; ++q) {
        const int2 ab = b.rot_ab[mg.lo + q];
        const double2 cs = b.rot_cs[mg.lo + q];
        double* pa = Z + row + (size_t)N * ab.x;
        double* pb = Z + row + (size_t)N * ab.y;
        const double za = *pa, zb = *pb;
        *pa = cs.x * za + cs.y * zb;
        *pb = -cs.y * za + cs.x * zb;
    }
}

// Roots of 1 + rho sum_i z_i^2 / (delta_i - lambda): one wave per root, the
// poles of the merge staged in LDS.
__global__ __launch_bounds__(256) void k_dc_secular(const DcMerge* __restrict__ plan, DcBuf b) {
    __shared__ double sd[4096];
    __shared__ double sz[4096];
    const DcMerge mg = plan[blockIdx.y];
    const int k = b.mk[mg.id];
    if ((int)blockIdx.x * 4 >= k) return;
    const int lo = mg.lo;
    for (int i = threadIdx.x; i < k; i += 256) {
        sd[i] = b.ndv[lo + i];
        const double z = b.ndz[lo + i];
        sz[i] = z * z;
    }
    __syncthreads();
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (j >= k) return;
    const double rho = b.mrho[mg.id];
    double zs = 0.0;
    for (int i = lane; i < k; i += 64) zs += sz[i];
    zs = wave_sum(zs);
    int o;
    double sgn, lo_s, hi_s;
    if (j < k - 1) {
        const double h = sd[j + 1] - sd[j];
        double f = 0.0;
        for (int i = lane; i < k; i += 64) f += sz[i] / ((sd[i] - sd[j]) - 0.5 * h);
        f = 1.0 + rho * wave_sum(f);
        const double den = 1.0 + 2.0 * rho * zs / h;
        if (f >= 0.0) { o = j; sgn = 1.0; lo_s = rho * sz[j] / den; }
        else { o = j + 1; sgn = -1.0; lo_s = rho * sz[j + 1] / den; }
        hi_s = 0.5 * h;
    } else {
        o = j;
        sgn = 1.0;
        hi_s = rho * zs;
        lo_s = 0.5 * rho * sz[j];
    }
    lo_s = fmin(lo_s, hi_s);
    const double dor = sd[o];
    for (int it = 0; it < 400; ++it) {
        const double mid = (lo_s > 0.0 && hi_s > 64.0 * lo_s) ? sqrt(lo_s * hi_s)
                         : (lo_s > 0.0 ? 0.5 * (lo_s + hi_s) : 0.5 * hi_s);
        if (!(mid > lo_s && mid < hi_s)) break;
        const double tau = sgn * mid;
        double g = 0.0;
        for (int i = lane; i < k; i += 64) g += sz[i] / ((sd[i] - dor) - tau);
        g = 1.0 + rho * wave_sum(g);
        if ((g >= 0.0) == (sgn > 0.0)) hi_s = mid;
        else lo_s = mid;
    }
    if (lane == 0) {
        const double tau = sgn * 0.5 * (lo_s + hi_s);
        b.taus[lo + j] = tau;
        b.orig[lo + j] = o;
        b.lam[lo + j] = dor + tau;
    }
}

// zhat_i^2 = (lambda_i - delta_i)/rho * prod_{j != i} (lambda_j - delta_i) / (delta_j - delta_i)
__global__ __launch_bounds__(256) void k_dc_zhat(const DcMerge* __restrict__ plan, DcBuf b) {
    __shared__ double sd[4096];
    const DcMerge mg = plan[blockIdx.y];
    const int k = b.mk[mg.id];
    if ((int)blockIdx.x * 4 >= k) return;
    const int lo = mg.lo;
    for (int i = threadIdx.x; i < k; i += 256) sd[i] = b.ndv[lo + i];
    __syncthreads();
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= k) return;
    const double rho = b.mrho[mg.id];
    const double di = sd[i];
    double p = 1.0;
    for (int q = lane; q < k; q += 64) {
        const double lq = b.taus[lo + q] - (di - sd[b.orig[lo + q]]);   // lambda_q - delta_i
        p *= q == i ? lq / rho : lq / (sd[q] - di);
    }
    p = wave_prod(p);
    if (lane == 0) b.zh[lo + i] = copysign(sqrt(fmax(p, 0.0)), b.ndz[lo + i]);
}

// U[:, j] = zhat / (delta - lambda_j), normalised (one wave per column).
__global__ __launch_bounds__(256) void k_dc_vec(const DcMerge* __restrict__ plan, int N, double* __restrict__ U,
                                                DcBuf b) {
    __shared__ double sd[4096];
    __shared__ double sz[4096];
    const DcMerge mg = plan[blockIdx.y];
    const int k = b.mk[mg.id];
    if ((int)blockIdx.x * 4 >= k) return;
    const int lo = mg.lo;
    for (int i = threadIdx.x; i < k; i += 256) { sd[i] = b.ndv[lo + i]; sz[i] = b.zh[lo + i]; }
    __syncthreads();
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (j >= k) return;
    const double tau = b.taus[lo + j], dor = sd[b.orig[lo + j]];
    double s = 0.0;
    for (int i = lane; i < k; i += 64) {
        const double u = sz[i] / ((sd[i] - dor) - tau);
        s += u * u;
    }
    s = wave_sum(s);
    const double inv = 1.0 / sqrt(s);
    double* col = U + lo + (size_t)N * (lo + j);
    for (int i = lane; i < k; i += 64) col[i] = sz[i] / ((sd[i] - dor) - tau) * inv;
}

// Z2[lo.., lo + j] = Z[lo.., ndc[i]] U[i, j] over the non-deflated columns.
__global__ __launch_bounds__(256) void k_dc_gemm(const DcMerge* __restrict__ plan, int N,
                                                 const double* __restrict__ Z, const double* __restrict__ U,
                                                 double* __restrict__ Z2, DcBuf b) {
    const DcMerge mg = plan[blockIdx.z];
    const int k = b.mk[mg.id], n = mg.n1 + mg.n2, lo = mg.lo;
    const int m0 = blockIdx.x * ZBM, n0 = blockIdx.y * ZBN;
    if (m0 >= n || n0 >= k) return;
    dgemm_tile<double, true>(n, k, k, Z + lo, N, b.ndc + lo, U + lo + (size_t)N * lo, N,
                             Z2 + lo + (size_t)N * lo, N, m0, n0);
}

// Deflated columns after the roots' columns: Z2[lo.., lo + k + u] = Z[lo.., dfc[u]].
__global__ __launch_bounds__(256) void k_dc_defl(const DcMerge* __restrict__ plan, int N,
                                                 const double* __restrict__ Z, double* __restrict__ Z2, DcBuf b) {
    const DcMerge mg = plan[blockIdx.y];
    const int k = b.mk[mg.id], n = mg.n1 + mg.n2, lo = mg.lo;
    const int u = blockIdx.x;
    if (u >= n - k) return;
    const double* src = Z + (size_t)N * b.dfc[lo + u] + lo;
    double* dst = Z2 + (size_t)N * (lo + k + u) + lo;
    for (int r = threadIdx.x; r < n; r += 256) dst[r] = src[r];
}

// All n eigenvalues of the merge (roots, then deflated values) in ascending
// order (bitonic, ties by position); perm[r] is the Z2 column of the r-th.
__global__ __launch_bounds__(1024) void k_dc_sort(const DcMerge* __restrict__ plan, DcBuf b) {
    __shared__ double sv[4096];
    __shared__ int si[4096];
    const DcMerge mg = plan[blockIdx.x];
    const int k = b.mk[mg.id], n = mg.n1 + mg.n2, lo = mg.lo;
    int P = 1;
    while (P < n) P <<= 1;
    for (int t = threadIdx.x; t < P; t += 1024) {
        si[t] = t;
        sv[t] = t < k ? b.lam[lo + t] : (t < n ? b.dfv[lo + t - k] : INFINITY);
    }
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < P; t += 1024) {
                const int pr = t ^ stride;
                if (pr > t) {
                    const bool up = (t & size) == 0;
                    const double a = sv[t], c = sv[pr];
                    const int ia = si[t], ic = si[pr];
                    const bool gt = a > c || (a == c && ia > ic);
                    if (gt == up) { sv[t] = c; sv[pr] = a; si[t] = ic; si[pr] = ia; }
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < n; t += 1024) {
        b.dv[lo + t] = sv[t];
        b.perm[lo + t] = lo + si[t];
    }
}

__global__ __launch_bounds__(256) void k_dc_perm(const DcMerge* __restrict__ plan, int N, double* __restrict__ Z,
                                                 const double* __restrict__ Z2, DcBuf b) {
    const DcMerge mg = plan[blockIdx.y];
    const int n = mg.n1 + mg.n2, lo = mg.lo;
    const int r = blockIdx.x;
    if (r >= n) return;
    const double* src = Z2 + (size_t)N * b.perm[lo + r] + lo;
    double* dst = Z + (size_t)N * (lo + r) + lo;
    for (int q = threadIdx.x; q < n; q += 256) dst[q] = src[q];
}

// --------------------------------------------------- back-transformation
// Y = [v_j0 .. v_j0+nb-1] (N x kBtNb, zero-padded) from the reflectors below the diagonal.
// The reflectors in place: G[i, j] <- 0 for i <= j, G[j+1, j] <- 1 (v_j's
// leading entry; the tridiagonalisation leaves alpha there), and column j <- 0
// where tau_j = 0 (no reflection), so that G's columns j0 .. j0+63 are the
// block's Y.
__global__ __launch_bounds__(256) void k_bt_mask(double2* __restrict__ G, int ldg, int N,
                                                 const double2* __restrict__ tau) {
    const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
    if (i >= N) return;
    const double2 t = j < N - 1 ? tau[j] : make_double2(0.0, 0.0);
    if (i <= j || (t.x == 0.0 && t.y == 0.0)) G[i + (size_t)ldg * j] = make_double2(0.0, 0.0);
    else if (i == j + 1) G[i + (size_t)ldg * j] = make_double2(1.0, 0.0);
}

// P = (X Y) T for H_j0 .. H_j0+nb-1 = I - Y T Y^H without forming T: T^{-1} is
// the strict upper triangle of S = Y^H Y with 1/tau_i on its diagonal (a
// reflector with tau = 0 has its column of Y replaced by zero), so every row
// of P solves p T^{-1} = (X Y)_row by forward substitution,
//   p_i = tau_i ((X Y)_i - sum_{q<i} p_q S[q][i]).
// ADJ: P = (X Y) T^H for the block's adjoint I - Y T^H Y^H; (T^H)^{-1} is the
// strict lower triangle of S (S is Hermitian) with 1/conj(tau_i) on its
// diagonal, so by backward substitution
//   p_i = conj(tau_i) ((X Y)_i - sum_{q>i} p_q S[q][i]).
// One wave per row of X, lane q holding entry q; the split-K partials of X Y
// are summed on the way.  Column by column: p_c is final once the earlier
// (later, for ADJ) columns are subtracted; it is broadcast from lane c and
// p_c S[c][l] is subtracted from the lanes still to come.
template <bool ADJ>
__global__ __launch_bounds__(256) void k_bt_solve(const double2* __restrict__ Ppart, int splits, int m,
                                                  const double2* __restrict__ S, const double2* __restrict__ tau,
                                                  int j0, int nbb, double2* __restrict__ P) {
    __shared__ double2 Ss[kBtNb][kBtNb + 1];
    __shared__ double2 ts[kBtNb];
    {
        static_assert(kBtNb == 64, "the block load covers 64 x 64");
        double2 v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = S[threadIdx.x + 256 * u];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int q = (int)threadIdx.x + 256 * u;
            Ss[q & 63][q >> 6] = v[u];
        }
    }
    if (threadIdx.x < kBtNb) {
        double2 tc = (int)threadIdx.x < nbb ? tau[j0 + threadIdx.x] : make_double2(0.0, 0.0);
        if (ADJ) tc.y = -tc.y;
        ts[threadIdx.x] = tc;
    }
    __syncthreads();
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= m) return;
    double2 b = make_double2(0.0, 0.0);
    for (int z = 0; z < splits; ++z) {
        const double2 v = Ppart[(size_t)z * m * kBtNb + i + (size_t)m * lane];
        b.x += v.x;
        b.y += v.y;
    }
    for (int k = 0; k < nbb; ++k) {
        const int c = ADJ ? nbb - 1 - k : k;
        const double2 pc = zmul(ts[c], make_double2(lane_bcast(b.x, c), lane_bcast(b.y, c)));
        double2 sc = Ss[c][lane];
        if (!(ADJ ? lane < c : (lane > c && lane < nbb))) sc = make_double2(0.0, 0.0);
        const double2 t = zmul(pc, sc);
        b.x = lane == c ? pc.x : b.x - t.x;
        b.y = lane == c ? pc.y : b.y - t.y;
    }
    P[i + (size_t)m * lane] = lane < nbb ? b : make_double2(0.0, 0.0);
}

// ------------------------------------------------ Gram check of the start
// d[i] = G[i][i] (real), info->gram_trace = sum of them; clears the measure.
__global__ __launch_bounds__(256) void k_gram_diag(const double2* __restrict__ G, int ld, int N,
                                                   double* __restrict__ d, DevInfo* __restrict__ info) {
    __shared__ double red[4];
    double t = 0.0;
    for (int i = threadIdx.x; i < N; i += 256) {
        const double v = G[i + (size_t)ld * i].x;
        d[i] = v;
        t += v;
    }
    t = block_sum<256>(t, red);
    if (threadIdx.x == 0) {
        info->gram_trace = t;
        info->offmax_bits = 0ull;
    }
}

// Largest |g_ij| / sqrt(g_ii g_jj) over the pairs of columns above the rounding
// floor (g_ii > zrel2 * trace G; lower triangle), as the Jacobi sweeps measure it, folded into
// info->offmax_bits (non-negative doubles order like their bit patterns).
__global__ __launch_bounds__(256) void k_gram_offmax(const double2* __restrict__ G, int ld, int N, double zrel2,
                                                     const double* __restrict__ d, DevInfo* __restrict__ info) {
    const double floor2 = zrel2 * info->gram_trace;
    const int j = blockIdx.y;
    const double gjj = d[j];
    double mx = 0.0;
    if (gjj > floor2)
        for (int i = j + 1 + blockIdx.x * 256 + threadIdx.x; i < N; i += gridDim.x * 256) {
            const double gii = d[i];
            if (gii > floor2) {
                const double2 g = G[i + (size_t)ld * j];
                mx = fmax(mx, sqrt(g.x * g.x + g.y * g.y) / sqrt(gii * gjj));
            }
        }
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0 && mx > 0.0)
        atomicMax(&info->offmax_bits, (unsigned long long)__double_as_longlong(mx));
}

// ------------------------------------------------ Cholesky QR re-gauge
// Exact re-gauge of a centre move ("Note added": the orthogonality centre is
// moved by QR): A (m x r) = Q R with Q an isometry, by shifted Cholesky QR
// followed by two plain Cholesky QR passes, all in FP64.  The first pass
// factors A^H A + s I with s = 11 (m r + r (r+1)) u ||A||_F^2, which keeps the
// Cholesky factorisation defined for condition numbers up to about 1/u and
// leaves Q_1 with condition number below about 1/sqrt(u); the next two passes
// make it orthonormal to working accuracy.  R = R_3 R_2 R_1 (upper).

// G[i][i] += coef * trace(G) (one work-group); clears the failure flag.
__global__ __launch_bounds__(256) void k_qr_shift(double2* __restrict__ G, int ldg, int r, double coef,
                                                  DevInfo* __restrict__ info) {
    __shared__ double red[4];
    double t = 0.0;
    for (int i = threadIdx.x; i < r; i += 256) t += G[i + (size_t)ldg * i].x;
    t = block_sum<256>(t, red);
    for (int i = threadIdx.x; i < r; i += 256) G[i + (size_t)ldg * i].x += coef * t;
    if (threadIdx.x == 0) {
        info->qr_shift = coef * t;
        info->qr_fail = 0;
    }
}

// Upper Cholesky factor of the kb x kb diagonal block at (k0, k0), in place (one
// work-group, the block in LDS).  A pivot at or below its bound sets
// info->qr_fail and is replaced by a tiny positive value, so that the pass still
// ends with finite data.  Bounds by pass kind:
//   kQrShifted  half the shift, which every pivot of the shifted Gram exceeds;
//   kQrAfterShift  1e-14: Q_1 conditioned beyond 1e7, past Cholesky QR twice;
//   kQrFinal    1/2: the Gram of a nearly orthonormal Q;
//   kQrPlain    1e-12 of the column's own squared norm (diag0): the column is
//               independent of the earlier ones to 1e-6 in angle, so one more
//               pass makes Q orthonormal.
// The kb x kb block of G at (k0, k0) into LDS (64 x 65), every load issued
// before the first LDS store so that their latencies overlap.
__device__ __forceinline__ void load_block64(double2 (*Bs)[65], const double2* __restrict__ G, int ldg, int k0,
                                             int kb) {
    double2 v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int q = (int)threadIdx.x + 256 * u, i = q & 63, jj = q >> 6;
        v[u] = (i < kb && jj < kb) ? G[(k0 + i) + (size_t)ldg * (k0 + jj)] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int q = (int)threadIdx.x + 256 * u;
        Bs[q & 63][q >> 6] = v[u];
    }
}

// G[i, j] = sum over z of P_z[i, j] (P_z r x r, stride r, one after the other),
// on the 64 x 64 tiles on or above the diagonal, partials added in order.
__global__ __launch_bounds__(256) void k_sum_upper(const double2* __restrict__ P, int splits, int r,
                                                   double2* __restrict__ G, int ldg) {
    const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
    if (i >= r || (i >> 6) > (j >> 6)) return;
    const size_t rr = (size_t)r * r;
    double2 acc = P[i + (size_t)r * j];
    for (int z = 1; z < splits; ++z) {
        const double2 v = P[rr * z + i + (size_t)r * j];
        acc.x += v.x;
        acc.y += v.y;
    }
    G[i + (size_t)ldg * j] = acc;
}

enum { kQrShifted = 0, kQrAfterShift = 1, kQrFinal = 2, kQrPlain = 3 };
__global__ __launch_bounds__(256) void k_chol_diag(double2* __restrict__ G, int ldg, int k0, int kb, int pass,
                                                   const double* __restrict__ diag0,
                                                   DevInfo* __restrict__ info) {
    // Right-looking, one barrier per step, the trailing rows in registers: row
    // p lives in wave p % 4 (slot p / 4), lane l holding column l.  At step i
    // the owner of row i reads it from LDS, where it published it in the step
    // before, forms row i of R and stores it there for good; after the barrier
    // every wave subtracts conj(R[i][p]) R[i][l] from its rows i < p <= l and
    // the owner of row i+1 publishes that row.  Register slots are only ever
    // addressed by compile-time indices.
    __shared__ double2 B[64][65];
    load_block64(B, G, ldg, k0, kb);
    __syncthreads();
    const double floor_piv = 1e-300;
    const double bound = pass == kQrShifted ? 0.5 * info->qr_shift
                       : pass == kQrAfterShift ? 1e-14 : pass == kQrFinal ? 0.5 : 0.0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // the plain pass's per-column bounds, loaded once (lane l: column l), so
    // that no step waits on global memory
    const double d0 = (pass == kQrPlain && lane < kb) ? diag0[k0 + lane] : 0.0;
    double2 b[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) b[u] = B[w + 4 * u][lane];
    for (int i = 0; i < kb; ++i) {
        if (w == (i & 3)) {
            double2 r = B[i][lane];
            const double piv = lane_bcast(r.x, i);
            const double bi = pass == kQrPlain ? 1e-12 * lane_bcast(d0, i) : bound;
            if (lane == 0 && !(piv > bi)) info->qr_fail = 1;
            const double dii = sqrt(fmax(piv, floor_piv));
            const double inv = 1.0 / dii;
            if (lane > i) r = make_double2(r.x * inv, r.y * inv);
            else if (lane == i) r = make_double2(dii, 0.0);
            B[i][lane] = r;
        }
        __syncthreads();
        const double2 ril = B[i][lane];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int p = w + 4 * u;
            const double2 t = zcmul(B[i][p], ril);
            if (p > i && p <= lane) b[u] = make_double2(b[u].x - t.x, b[u].y - t.y);
            if (p == i + 1) B[p][lane] = b[u];
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kb * kb; q += 256) {
        const int i = q % kb, j = q / kb;
        G[(k0 + i) + (size_t)ldg * (k0 + j)] = i <= j ? B[i][j] : make_double2(0.0, 0.0);
    }
}

// Triangular substitution across the lanes of a wave for NR right-hand sides
// at once, lane l holding entry l of each (l < kb), R upper triangular with a
// real diagonal in LDS (R[i][j] = Rk[i][j]), rinv[i] = 1 / R[i][i]:
//   CONJ = false   x R = b     x_l = (b_l - sum_{c<l} x_c R[c][l]) / R[l][l]
//   CONJ = true    R^H x = b   x_l = (b_l - sum_{c<l} conj(R[c][l]) x_c) / R[l][l]
// Column by column: x_c is final once the earlier columns are subtracted; it
// is broadcast from lane c and subtracted from the later lanes.
template <bool CONJ, int NR>
__device__ __forceinline__ void lane_subst(double2 (&b)[NR], const double2 (*Rk)[65], const double* rinv, int kb,
                                           int lane) {
    // no branches: the row of R is masked to the lanes still to come, and the
    // solved lane takes x_c by a select
    for (int c = 0; c < kb; ++c) {
        double2 rc = Rk[c][lane < kb ? lane : 0];
        if (lane <= c) rc = make_double2(0.0, 0.0);
        const double ri = rinv[c];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const double2 xc = make_double2(lane_bcast(b[k].x, c) * ri, lane_bcast(b[k].y, c) * ri);
            const double2 t = CONJ ? zcmul(rc, xc) : zmul(xc, rc);
            b[k].x = lane == c ? xc.x : b[k].x - t.x;
            b[k].y = lane == c ? xc.y : b[k].y - t.y;
        }
    }
}

constexpr int kSubstRows = 4;   // right-hand sides per wave of the substitution kernels

// Row block of R right of the diagonal block: R[k, j] = R_kk^{-H} G[k, j] for the
// columns j in [k0 + kb, r); kSubstRows columns per wave.
__global__ __launch_bounds__(256) void k_chol_row(double2* __restrict__ G, int ldg, int k0, int kb, int r) {
    __shared__ double2 Rk[64][65];
    __shared__ double rinv[64];
    load_block64(Rk, G, ldg, k0, kb);
    if (threadIdx.x < kb) rinv[threadIdx.x] = 1.0 / G[(k0 + threadIdx.x) + (size_t)ldg * (k0 + threadIdx.x)].x;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int j0 = k0 + kb + (blockIdx.x * 4 + (threadIdx.x >> 6)) * kSubstRows;
    if (j0 >= r) return;
    double2 x[kSubstRows];
#pragma unroll
    for (int k = 0; k < kSubstRows; ++k) {
        const int j = j0 + k;
        x[k] = (lane < kb && j < r) ? G[(k0 + lane) + (size_t)ldg * j] : make_double2(0.0, 0.0);
    }
    lane_subst<true, kSubstRows>(x, Rk, rinv, kb, lane);
#pragma unroll
    for (int k = 0; k < kSubstRows; ++k) {
        const int j = j0 + k;
        if (lane < kb && j < r) G[(k0 + lane) + (size_t)ldg * j] = x[k];
    }
}

// Columns k0 .. k0+kb of Q (A is the whole m x r matrix): q_row R_kk = a_row (the
// earlier blocks already subtracted); kSubstRows rows per wave.
__global__ __launch_bounds__(256) void k_qr_rowsolve(double2* __restrict__ A, int lda, int m,
                                                     const double2* __restrict__ G, int ldg, int k0, int kb) {
    __shared__ double2 Rk[64][65];
    __shared__ double rinv[64];
    load_block64(Rk, G, ldg, k0, kb);
    if (threadIdx.x < kb) rinv[threadIdx.x] = 1.0 / G[(k0 + threadIdx.x) + (size_t)ldg * (k0 + threadIdx.x)].x;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int i0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * kSubstRows;
    if (i0 >= m) return;
    double2 x[kSubstRows];
#pragma unroll
    for (int k = 0; k < kSubstRows; ++k) {
        const int i = i0 + k;
        x[k] = (lane < kb && i < m) ? A[i + (size_t)lda * (k0 + lane)] : make_double2(0.0, 0.0);
    }
    lane_subst<false, kSubstRows>(x, Rk, rinv, kb, lane);
#pragma unroll
    for (int k = 0; k < kSubstRows; ++k) {
        const int i = i0 + k;
        if (lane < kb && i < m) A[i + (size_t)lda * (k0 + lane)] = x[k];
    }
}

// diag0[i] = G[i][i] (the columns' squared norms, for the plain pass's bounds);
// clears the failure flag.
__global__ __launch_bounds__(256) void k_qr_diag0(const double2* __restrict__ G, int ldg, int r,
                                                  double* __restrict__ diag0, DevInfo* __restrict__ info) {
    for (int i = threadIdx.x; i < r; i += 256) diag0[i] = G[i + (size_t)ldg * i].x;
    if (threadIdx.x == 0) info->qr_fail = 0;
}

// Rp (r x r, stride r) = the upper triangle of G.
__global__ __launch_bounds__(256) void k_qr_triu(const double2* __restrict__ G, int ldg, int r,
                                                 double2* __restrict__ Rp) {
    const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
    if (i < r) Rp[i + (size_t)r * j] = i <= j ? G[i + (size_t)ldg * j] : make_double2(0.0, 0.0);
}

template <typename T>
__global__ __launch_bounds__(256) void k_from_f64(const double2* __restrict__ Xd, int ldd, int m,
                                                  C2<T>* __restrict__ X, int ld) {
    const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
    if (i < m) X[i + (size_t)ld * j] = from_d2<T>(Xd[i + (size_t)ldd * j]);
}

// ------------------------------------------------------------ host plans
struct DcPlan {
    std::vector<int> level_off, level_cnt, level_nmax;
    DcMerge* dev = nullptr;   // all merges, level by level
};

int dc_build(int lo, int n, std::vector<std::vector<DcMerge>>& by_h) {
    if (n == 1) return 0;
    const int n1 = n / 2, n2 = n - n1;
    const int h = 1 + std::max(dc_build(lo, n1, by_h), dc_build(lo + n1, n2, by_h));
    if ((int)by_h.size() <= h) by_h.resize(h + 1);
    by_h[h].push_back({lo, n1, n2, 0});
    return h;
}

}  // namespace

struct HeevPlans {
    std::map<int, DcPlan> plans;
    ~HeevPlans() {
        for (auto& kv : plans)
            if (kv.second.dev) (void)hipFree(kv.second.dev);
    }
};

void* heev_plans_new() { return new HeevPlans(); }
void heev_plans_free(void* p) { delete (HeevPlans*)p; }

size_t heev_bytes(int m_max, int n_max) {
    if (n_max <= 0) return 0;
    const size_t N = n_max, ldx = (size_t)((m_max + 1) & ~1) + 8;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t b = 0;
    b += al(ldx * N * sizeof(double2));                         // Xd
    b += al((N + 8) * N * sizeof(double2));                     // G
    b += 2 * al(N * 2 * kTrdNb * sizeof(double2));              // VW, WV
    b += al((N / kHt + 2) * N * sizeof(double2));               // slots of the trailing product
    b += al((size_t)(N / kHt + 1) * (N / kHt + 2) / 2 * sizeof(double2));   // tiles' parts of u^H G u
    b += al(2 * kPart * sizeof(double));                        // norm partials (two halves)
    b += al((size_t)2 * kPart * 2 * kTrdNb * sizeof(double2));  // dot partials (two halves)
    b += al((1 + 2 * kTrdNb) * sizeof(double2));                // a column's reduced sums
    b += al(N * sizeof(double2));                               // tau
    b += 2 * al(N * sizeof(double));                            // d, e
    b += al((N / kBtNb + 1) * kBtNb * kBtNb * sizeof(double2)); // S = Y^H Y of every block
    const size_t splits = (N + kSplitK - 1) / kSplitK;
    b += al(splits * std::max<size_t>(ldx, kBtNb) * kBtNb * sizeof(double2));   // split-K partials
    b += al(ldx * kBtNb * sizeof(double2));                     // P
    b += 3 * al(N * N * sizeof(double));                        // Z, Z2, U
    b += 9 * al(N * sizeof(double));                            // dv ds dz ndv ndz dfv taus lam zh
    b += 5 * al(N * sizeof(int));                               // dcol ndc dfc orig perm
    b += al(N * sizeof(int2)) + al(N * sizeof(double2));        // rotations
    b += 2 * al(N * sizeof(int)) + al(N * sizeof(double));      // per-merge k, rotations, rho
    return b;
}

void heev_carve(char* p, int m_max, int n_max, HeevWork& w) {
    const size_t N = n_max, ldx = (size_t)((m_max + 1) & ~1) + 8;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    auto take = [&](size_t bytes) { char* q = p; p += al(bytes); return q; };
    w.cap_m = m_max;
    w.cap_n = n_max;
    w.Xd = (double2*)take(ldx * N * sizeof(double2));
    w.G = (double2*)take((N + 8) * N * sizeof(double2));
    w.VW = (double2*)take(N * 2 * kTrdNb * sizeof(double2));
    w.WV = (double2*)take(N * 2 * kTrdNb * sizeof(double2));
    w.ypart = (double2*)take((N / kHt + 2) * N * sizeof(double2));
    w.upart = (double2*)take((size_t)(N / kHt + 1) * (N / kHt + 2) / 2 * sizeof(double2));
    w.part = (double*)take(2 * kPart * sizeof(double));
    w.pdot = (double2*)take((size_t)2 * kPart * 2 * kTrdNb * sizeof(double2));
    w.pfin = (double2*)take((1 + 2 * kTrdNb) * sizeof(double2));
    w.tau = (double2*)take(N * sizeof(double2));
    w.d = (double*)take(N * sizeof(double));
    w.e = (double*)take(N * sizeof(double));
    w.Sall = (double2*)take((N / kBtNb + 1) * kBtNb * kBtNb * sizeof(double2));
    const size_t splits = (N + kSplitK - 1) / kSplitK;
    w.Cpart = (double2*)take(splits * std::max<size_t>(ldx, kBtNb) * kBtNb * sizeof(double2));
    w.P = (double2*)take(ldx * kBtNb * sizeof(double2));
    w.Z = (double*)take(N * N * sizeof(double));
    w.Z2 = (double*)take(N * N * sizeof(double));
    w.U = (double*)take(N * N * sizeof(double));
    double** dbl[] = {&w.dv, &w.ds, &w.dz, &w.ndv, &w.ndz, &w.dfv, &w.taus, &w.lam, &w.zh};
    for (double** q : dbl) *q = (double*)take(N * sizeof(double));
    int** ints[] = {&w.dcol, &w.ndc, &w.dfc, &w.orig, &w.perm};
    for (int** q : ints) *q = (int*)take(N * sizeof(int));
    w.rot_ab = (int2*)take(N * sizeof(int2));
    w.rot_cs = (double2*)take(N * sizeof(double2));
    w.mk = (int*)take(N * sizeof(int));
    w.mnrot = (int*)take(N * sizeof(int));
    w.mrho = (double*)take(N * sizeof(double));
}

namespace {

const DcPlan& dc_plan(HeevPlans& hp, int N) {
    auto it = hp.plans.find(N);
    if (it != hp.plans.end()) return it->second;
    std::vector<std::vector<DcMerge>> by_h;
    dc_build(0, N, by_h);
    DcPlan pl;
    std::vector<DcMerge> all;
    for (size_t h = 1; h < by_h.size(); ++h) {
        pl.level_off.push_back((int)all.size());
        pl.level_cnt.push_back((int)by_h[h].size());
        int nmax = 0;
        for (DcMerge m : by_h[h]) {
            m.id = (int)all.size();
            nmax = std::max(nmax, m.n1 + m.n2);
            all.push_back(m);
        }
        pl.level_nmax.push_back(nmax);
    }
    if (!all.empty()) {
        if (hipMalloc((void**)&pl.dev, all.size() * sizeof(DcMerge)) != hipSuccess ||
            hipMemcpy(pl.dev, all.data(), all.size() * sizeof(DcMerge), hipMemcpyHostToDevice) != hipSuccess)
            throw HeevFailure{"divide-and-conquer plan upload"};
    }
    return hp.plans.emplace(N, std::move(pl)).first->second;
}

}  // namespace

// Eigenvalues (ascending, w.dv) and eigenvectors (w.Z, N x N, ld N) of the
// Hermitian G (w.G, ld w.ldg), which is overwritten by its reflectors.
void heev_run(int N, HeevWork& w, Profiler& pf, hipStream_t st) {
    const int ldg = N + 8;
    if (N > 64 * kPart) throw HeevFailure{"tridiagonalisation row chunks"};
    // ---- tridiagonalisation (lower triangle of G only): the trailing
    // matrix-vector products are booked as K_TRIDIAG, the vector kernels and
    // the rank-2 nb panel updates as K_TRDAUX
    for (int j0 = 0; j0 < N - 1; j0 += kTrdNb) {
        const int nbb = std::min(kTrdNb, N - 1 - j0);
        const double pn = (double)N * 2 * kTrdNb;
        // every step kernel writes its panel column of V and W on all N rows
        // (zero above the reflector), so only a last, partial panel leaves
        // columns of the buffers that the rank update reads unwritten
        if (nbb < kTrdNb) {
            launch_booked(pf, K_TRDAUX, 0.0, 32.0 * pn, k_fill_z, dim3(64), dim3(256), 0, st, w.VW, (size_t)pn);
            launch_booked(pf, K_TRDAUX, 0.0, 32.0 * pn, k_fill_z, dim3(64), dim3(256), 0, st, w.WV, (size_t)pn);
        }
        launch_booked(pf, K_TRDAUX, 0.0, 16.0 * (N - j0), k_trd_colnorm, dim3(kPart), dim3(256), 0, st,
                      (const double2*)w.G, ldg, N, j0, w.part + (j0 & 1) * kPart);
        for (int c = 0; c < nbb; ++c) {
            const int j = j0 + c, len = N - j - 1;
            const int groups = (len + kHt - 1) / kHt;   // 64-row blocks of the trailing part
            const int ntiles = groups * (groups + 1) / 2;
            const int cur = j & 1, nxt = cur ^ 1;   // halves of the double-buffered partial sums
            launch_booked(pf, K_TRIDIAG, 8.0 * (double)len * len, 8.0 * (double)len * (len + 1), k_trd_hemv,
                          dim3(ntiles + 1), dim3(256), 0, st, (const double2*)w.G, ldg, N, j, w.ypart, w.upart, c,
                          (const double*)(w.part + cur * kPart), (const double2*)(w.pdot + cur * kPart * 2 * kTrdNb),
                          w.pfin);
            launch_booked(pf, K_TRDAUX, 16.0 * len * (3.0 * c + 4.0),
                          16.0 * ((double)len * (groups + 1) / kPart * kPart + len * (4.0 * c + 6.0) + ntiles),
                          k_trd_step, dim3(kPart), dim3(64 * kStepG), 0, st, w.G, ldg, N, j, c, (int)(c + 1 < nbb),
                          (const double2*)w.ypart, (const double2*)w.upart, w.VW, w.WV, (const double2*)w.pfin,
                          w.part + nxt * kPart, w.pdot + nxt * kPart * 2 * kTrdNb, w.tau, w.d, w.e);
        }
        const int k0 = j0 + nbb;
        zgemm<0, 1, 3>(N - k0, N - k0, 2 * kTrdNb, w.VW + k0, N, w.WV + k0, N, w.G + k0 + (size_t)ldg * k0, ldg,
                       st, 1, 0, 0, 0, 0, &pf, K_TRDAUX);
    }
    hipLaunchKernelGGL(k_trd_last, dim3(1), dim3(64), 0, st, (const double2*)w.G, ldg, N, w.d);

    // ---- divide and conquer
    pf.begin(st);
    const DcPlan& pl = dc_plan(*(HeevPlans*)w.plans, N);
    {
        const size_t nn = (size_t)N * N;
        hipLaunchKernelGGL(k_dc_init, dim3((unsigned)std::min<size_t>(4096, (nn + 255) / 256)), dim3(256), 0, st,
                           N, (const double*)w.d, (const double*)w.e, w.dv, w.Z);
    }
    DcBuf b{w.dv, w.ds, w.dz, w.ndv, w.ndz, w.dfv, w.taus, w.lam, w.zh, w.dcol, w.ndc, w.dfc,
            w.orig, w.perm, w.rot_ab, w.rot_cs, w.mk, w.mnrot, w.mrho};
    for (size_t L = 0; L < pl.level_off.size(); ++L) {
        const DcMerge* mg = pl.dev + pl.level_off[L];
        const unsigned cnt = pl.level_cnt[L];
        const int nmax = pl.level_nmax[L];
        hipLaunchKernelGGL(k_dc_prep, dim3(cnt), dim3(1024), 0, st, mg, N, (const double*)w.e,
                           (const double*)w.Z, b);
        hipLaunchKernelGGL(k_dc_rot, dim3((nmax + 255) / 256, cnt), dim3(256), 0, st, mg, N, w.Z, b);
        const unsigned g4 = (nmax + 3) / 4;
        hipLaunchKernelGGL(k_dc_secular, dim3(g4, cnt), dim3(256), 0, st, mg, b);
        hipLaunchKernelGGL(k_dc_zhat, dim3(g4, cnt), dim3(256), 0, st, mg, b);
        hipLaunchKernelGGL(k_dc_vec, dim3(g4, cnt), dim3(256), 0, st, mg, N, w.U, b);
        const unsigned gt = (nmax + ZBM - 1) / ZBM;
        hipLaunchKernelGGL(k_dc_gemm, dim3(gt, gt, cnt), dim3(256), 0, st, mg, N, (const double*)w.Z,
                           (const double*)w.U, w.Z2, b);
        hipLaunchKernelGGL(k_dc_defl, dim3(nmax, cnt), dim3(256), 0, st, mg, N, (const double*)w.Z, w.Z2, b);
        hipLaunchKernelGGL(k_dc_sort, dim3(cnt), dim3(1024), 0, st, mg, b);
        hipLaunchKernelGGL(k_dc_perm, dim3(nmax, cnt), dim3(256), 0, st, mg, N, w.Z, (const double*)w.Z2, b);
    }
    pf.end(st, K_DC, 2.0 * (double)N * N * N, 24.0 * (double)N * N);
}

// X (rows x N, FP64, stride ldx) <- X Q_H, blocks of kBtNb reflectors in forward
// order: X[:, j0+1:] -= ((X[:, j0+1:] Y) T) Y^H with Y the block's reflectors and
// T its triangular factor (H_j0 .. H_j0+nb-1 = I - Y T Y^H).  ADJ: X <- X Q_H^H,
// the blocks' adjoints I - Y T^H Y^H in backward order.
template <bool ADJ>
static void apply_qh(double2* X, int rows, int ldx, int N, HeevWork& w, Profiler& pf, hipStream_t st) {
    const int ldg = N + 8;
    const int nblk = (N - 1 + kBtNb - 1) / kBtNb;
    // Y of every block in G itself, and S_b = Y_b^H Y_b of all blocks at once
    // (the blocks whose 64 columns lie inside G batched, a last partial one alone;
    // rows above a block are zero, so every product runs over all N rows)
    launch_booked(pf, K_BTAUX, 0.0, 8.0 * (double)N * N, k_bt_mask, dim3((N + 255) / 256, N), dim3(256), 0, st, w.G,
                  ldg, N, (const double2*)w.tau);
    const int nfull = std::min(nblk, N / kBtNb);
    const size_t sS = (size_t)kBtNb * kBtNb;
    zgemm<1, 0, 0>(kBtNb, kBtNb, N, w.G, ldg, w.G, ldg, w.Sall, kBtNb, st, nfull, 0, (size_t)ldg * kBtNb,
                   (size_t)ldg * kBtNb, sS, &pf, K_BTAUX);
    if (nfull < nblk) {
        const int j0 = nfull * kBtNb, nc = N - j0;
        zgemm<1, 0, 0>(nc, nc, N, w.G + (size_t)ldg * j0, ldg, w.G + (size_t)ldg * j0, ldg, w.Sall + sS * nfull,
                       kBtNb, st, 1, 0, 0, 0, 0, &pf, K_BTAUX);
    }
    for (int bk = 0; bk < nblk; ++bk) {
        const int b = ADJ ? nblk - 1 - bk : bk;
        const int j0 = b * kBtNb;
        const int nbb = std::min(kBtNb, N - 1 - j0);
        const int K = N - j0 - 1;                  // rows j0+1 .. N-1 of Y
        const int splits = (K + kSplitK - 1) / kSplitK;
        const double2* Ys = w.G + (j0 + 1) + (size_t)ldg * j0;
        // X Y (split-K), then P = (X Y) T (or T^H) by row-wise substitution
        zgemm<0, 0, 0>(rows, nbb, K, X + (size_t)ldx * (j0 + 1), ldx, Ys, ldg, w.Cpart, rows, st, splits, kSplitK,
                       (size_t)kSplitK * ldx, kSplitK, (size_t)rows * kBtNb, &pf, K_BACK);
        launch_booked(pf, K_BTAUX, 8.0 * rows * kBtNb * kBtNb / 2, 16.0 * rows * kBtNb * (splits + 1),
                      k_bt_solve<ADJ>, dim3((rows + 3) / 4), dim3(256), 0, st, (const double2*)w.Cpart, splits, rows,
                      (const double2*)(w.Sall + sS * b), (const double2*)w.tau, j0, nbb, w.P);
        // X[:, j0+1:] -= P Y^H
        zgemm<0, 1, 1>(rows, K, nbb, w.P, rows, Ys, ldg, X + (size_t)ldx * (j0 + 1), ldx, st, 1, 0, 0, 0, 0, &pf,
                       K_BACK);
    }
}

// M[r, i] = Z[i, N-1-r] (as complex): the last `keep` eigenvectors (largest
// eigenvalues first) as the rows of M (stride ldm).
__global__ __launch_bounds__(256) void k_top_rows(const double* __restrict__ Z, int N, int keep,
                                                  double2* __restrict__ M, int ldm) {
    const int r = blockIdx.x * 256 + threadIdx.x, i = blockIdx.y;
    if (r < keep) M[r + (size_t)ldm * i] = make_double2(Z[i + (size_t)N * (N - 1 - r)], 0.0);
}

// *rest = sum of the n smallest eigenvalues (ascending dv), negatives (rounding) as 0.
__global__ __launch_bounds__(256) void k_rest_weight(const double* __restrict__ dv, int n, double* rest) {
    __shared__ double red[4];
    double t = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) t += fmax(dv[i], 0.0);
    t = block_sum<256>(t, red);
    if (threadIdx.x == 0) *rest = t;
}

// X (m x N, storage T, stride ld) <- X Q_H Z for the Gram eigen-decomposition
// of X, all in FP64.  With keep < N only the eigenvectors of the keep largest
// eigenvalues are applied, X (m x keep) <- X (Q_H Z_keep): Q_H Z_keep =
// (Z_keep^T Q_H^H)^H is formed on the keep x N matrix M (the reflectors' cost
// falls with keep / m), and *rest (device) receives the sum of the other
// eigenvalues, the weight of the columns left out.  Returns the number of
// columns written (keep, or N when the subset does not fit the scratch).
// Throws HeevFailure on a HIP error.
template <typename T>
int heev_precondition(C2<T>* X, int m, int N, int ld, int keep, double* rest, HeevWork& w, Profiler& pf,
                      hipStream_t st) {
    if (N > w.cap_n || m > w.cap_m || N < 2) throw HeevFailure{"eigen-preconditioner capacity"};
    const int ldx = ((w.cap_m + 1) & ~1) + 8;
    const int ldg = N + 8;
    const int ldm = ((keep + 1) & ~1) + 8;
    // M lives in the divide-and-conquer scratch U, the FP64 product in Z2 (both
    // N x N doubles, free once the eigenvectors are in Z)
    const bool subset = keep < N && rest != nullptr && 2 * (size_t)ldm * N <= (size_t)N * N &&
                        2 * (size_t)m * keep <= (size_t)N * N;
    // ---- X -> FP64, Gram (lower triangle)
    launch_booked(pf, K_BTAUX, 0.0, (double)m * N * (sizeof(C2<T>) + 16.0), k_to_f64<T>, dim3((m + 255) / 256, N),
                  dim3(256), 0, st, (const C2<T>*)X, m, ld, w.Xd, ldx);
    zgemm<1, 0, 2>(N, N, m, w.Xd, ldx, w.Xd, ldx, w.G, ldg, st, 1, 0, 0, 0, 0, &pf, K_HGRAM);

    heev_run(N, w, pf, st);

    if (!subset) {
        // ---- X <- X Q_H
        apply_qh<false>(w.Xd, m, ldx, N, w, pf, st);
        // ---- X <- Xd Z (real view: 2m x N times N x N), rounded to the storage precision
        launch_booked(pf, K_HOUT, 4.0 * (double)m * N * N,
                      16.0 * (double)m * N + 8.0 * (double)N * N + (double)m * N * sizeof(C2<T>), k_dgemm<T>,
                      dim3((2 * m + ZBM - 1) / ZBM, (N + ZBN - 1) / ZBN), dim3(256), 0, st, 2 * m, N, N,
                      (const double*)w.Xd, 2 * ldx, (const double*)w.Z, N, (T*)X, 2 * ld);
        if (hipGetLastError() != hipSuccess) throw HeevFailure{"eigen-preconditioner launch"};
        w.n_runs += 1;
        return N;
    }
    double2* M = (double2*)w.U;
    double2* Xo = (double2*)w.Z2;
    launch_booked(pf, K_HOUT, 0.0, 24.0 * (double)keep * N, k_top_rows, dim3((keep + 255) / 256, N), dim3(256), 0, st,
                  (const double*)w.Z, N, keep, M, ldm);
    apply_qh<true>(M, keep, ldm, N, w, pf, st);
    // ---- X (m x keep) <- Xd M^H, rounded to the storage precision
    zgemm<0, 1, 0>(m, keep, N, w.Xd, ldx, M, ldm, Xo, m, st, 1, 0, 0, 0, 0, &pf, K_HOUT);
    launch_booked(pf, K_HOUT, 0.0, (double)m * keep * (16.0 + sizeof(C2<T>)), k_from_f64<T>,
                  dim3((m + 255) / 256, keep), dim3(256), 0, st, (const double2*)Xo, m, m, X, ld);
    launch_booked(pf, K_HOUT, 0.0, 8.0 * (N - keep), k_rest_weight, dim3(1), dim3(256), 0, st, (const double*)w.dv,
                  N - keep, rest);
    if (hipGetLastError() != hipSuccess) throw HeevFailure{"eigen-preconditioner launch"};
    w.n_runs += 1;
    return keep;
}

template int heev_precondition<double>(double2*, int, int, int, int, double*, HeevWork&, Profiler&, hipStream_t);
template int heev_precondition<float>(float2*, int, int, int, int, double*, HeevWork&, Profiler&, hipStream_t);

// Hermitian eigen-decomposition of a host matrix (tests): G row-major complex
// N x N (interleaved), values ascending, vectors as columns of V (row-major).
void heev_host(int N, const double* Gh, double* wh, double* Vh, HeevWork& w, Profiler& pf, hipStream_t st) {
    if (N > w.cap_n || N < 2) throw HeevFailure{"eigen-solver capacity"};
    const int ldg = N + 8;
    std::vector<double2> g((size_t)ldg * N);
    for (int r = 0; r < N; ++r)
        for (int c = 0; c < N; ++c) g[r + (size_t)ldg * c] = make_double2(Gh[2 * (r * N + c)], Gh[2 * (r * N + c) + 1]);
    if (hipMemcpyAsync(w.G, g.data(), g.size() * sizeof(double2), hipMemcpyHostToDevice, st) != hipSuccess)
        throw HeevFailure{"copy in"};
    heev_run(N, w, pf, st);
    // V = Q_H Z: apply the reflectors to Z (as complex) through the same right-multiplication
    // on X = I: Xd <- I, Xd <- Xd Q_H, V = Xd Z.
    const int ldx = ((w.cap_m + 1) & ~1) + 8;
    std::vector<double2> eye((size_t)ldx * N, make_double2(0.0, 0.0));
    for (int i = 0; i < N; ++i) eye[i + (size_t)ldx * i] = make_double2(1.0, 0.0);
    if (hipMemcpyAsync(w.Xd, eye.data(), eye.size() * sizeof(double2), hipMemcpyHostToDevice, st) != hipSuccess)
        throw HeevFailure{"copy in"};
    apply_qh<false>(w.Xd, N, ldx, N, w, pf, st);
    // V (complex, N x N, ld ldx) into G's storage
    {
        dim3 grid((2 * N + ZBM - 1) / ZBM, (N + ZBN - 1) / ZBN);
        hipLaunchKernelGGL((k_dgemm<double>), grid, dim3(256), 0, st, 2 * N, N, N, (const double*)w.Xd, 2 * ldx,
                           (const double*)w.Z, N, (double*)w.G, 2 * ldg);
    }
    if (hipGetLastError() != hipSuccess) throw HeevFailure{"launch"};
    std::vector<double> vals(N);
    if (hipMemcpyAsync(vals.data(), w.dv, N * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(g.data(), w.G, g.size() * sizeof(double2), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        throw HeevFailure{"copy out"};
    for (int i = 0; i < N; ++i) wh[i] = vals[i];
    for (int r = 0; r < N; ++r)
        for (int c = 0; c < N; ++c) {
            Vh[2 * (r * N + c)] = g[r + (size_t)ldg * c].x;
            Vh[2 * (r * N + c) + 1] = g[r + (size_t)ldg * c].y;
        }
}

// Q (m x r, storage T, stride ldq) and R (r x r, storage T, stride r) with A = Q R,
// A (m x r, storage T, stride lda); Q may overwrite A (it is written last).  All
// arithmetic in FP64.  First Cholesky QR twice; if a pivot of it falls below its
// bound (A too ill-conditioned), shifted Cholesky QR and two more passes from A
// again.  Returns false, with Q and R unwritten, if that too meets a pivot below
// its bound (A numerically rank-deficient).  Reads the flag back through the
// pinned info_host (synchronises the stream once or twice).
template <typename T>
bool cholqr3(const C2<T>* A, int m, int r, int lda, C2<T>* Q, int ldq, C2<T>* R, DevInfo* info,
             DevInfo* info_host, HeevWork& w, Profiler& pf, hipStream_t st) {
    if (r > w.cap_n || m > w.cap_m || r < 1 || 2 * (size_t)r * r > (size_t)w.cap_n * w.cap_n)
        throw HeevFailure{"Cholesky QR capacity"};
    const int ldx = ((w.cap_m + 1) & ~1) + 8;
    const int ldg = r + 8;
    double2* Ad = w.Xd;
    double2* Rt = nullptr;            // accumulated R (one of Z, U)
    double2* Rp = (double2*)w.Z2;     // this pass's R
    const double u = 1.1102230246251565e-16;
    std::function<void(int, int)> trsm = [&](int c0, int nc) {
        if (nc <= 64) {
            launch_booked(pf, K_QR, 4.0 * (double)m * nc * nc, 32.0 * (double)m * nc, k_qr_rowsolve,
                          dim3((m + 4 * kSubstRows - 1) / (4 * kSubstRows)), dim3(256), 0, st, Ad, ldx, m, (const double2*)w.G, ldg, c0, nc);
            return;
        }
        const int h = ((nc / 2 + 63) / 64) * 64;
        trsm(c0, h);
        zgemm<0, 0, 1>(m, nc - h, h, Ad + (size_t)ldx * c0, ldx, w.G + c0 + (size_t)ldg * (c0 + h), ldg,
                       Ad + (size_t)ldx * (c0 + h), ldx, st, 1, 0, 0, 0, 0, &pf, K_QR);
        trsm(c0 + h, nc - h);
    };
    // the Gram of a wide block has few output tiles (136 for r = 1024): its K
    // range is split over up to four launches' worth of work-groups, whose
    // partials go to whichever of Z, U holds no R factor, and summed in order
    const int gsplit = r >= 512 ? (int)std::min<size_t>(4, (size_t)w.cap_n * w.cap_n / (2 * (size_t)r * r)) : 1;
    auto pass_run = [&](int kind) {
        // the Cholesky factorisation reads the upper triangle only
        if (gsplit >= 2) {
            double2* part = Rt == (double2*)w.Z ? (double2*)w.U : (double2*)w.Z;
            const int kchunk = (((m + gsplit - 1) / gsplit) + 15) & ~15;
            const int nz = (m + kchunk - 1) / kchunk;
            zgemm<1, 0, 4>(r, r, m, Ad, ldx, Ad, ldx, part, r, st, nz, kchunk, (size_t)kchunk, (size_t)kchunk,
                           (size_t)r * r, &pf, K_QR);
            launch_booked(pf, K_QR, 0.0, 16.0 * (nz + 1.0) * r * r / 2, k_sum_upper, dim3((r + 255) / 256, r),
                          dim3(256), 0, st, (const double2*)part, nz, r, w.G, ldg);
        } else {
            zgemm<1, 0, 4>(r, r, m, Ad, ldx, Ad, ldx, w.G, ldg, st, 1, 0, 0, 0, 0, &pf, K_QR);
        }
        if (kind == kQrShifted)
            launch_booked(pf, K_QR, 0.0, 16.0 * r, k_qr_shift, dim3(1), dim3(256), 0, st, w.G, ldg, r,
                          11.0 * ((double)m * r + (double)r * (r + 1)) * u, info);
        if (kind == kQrPlain)
            launch_booked(pf, K_QR, 0.0, 24.0 * r, k_qr_diag0, dim3(1), dim3(256), 0, st, (const double2*)w.G, ldg, r,
                          w.dv, info);
        for (int k0 = 0; k0 < r; k0 += 64) {
            const int kb = std::min(64, r - k0), rest = r - k0 - kb;
            launch_booked(pf, K_QR, 0.0, 32.0 * kb * kb, k_chol_diag, dim3(1), dim3(256), 0, st, w.G, ldg, k0, kb,
                          kind, (const double*)w.dv, info);
            if (rest > 0) {
                launch_booked(pf, K_QR, 4.0 * kb * kb * rest, 32.0 * kb * rest, k_chol_row,
                              dim3((rest + 4 * kSubstRows - 1) / (4 * kSubstRows)),
                              dim3(256), 0, st, w.G, ldg, k0, kb, r);
                double2* Rrow = w.G + k0 + (size_t)ldg * (k0 + kb);
                zgemm<1, 0, 5>(rest, rest, kb, Rrow, ldg, Rrow, ldg, w.G + (k0 + kb) + (size_t)ldg * (k0 + kb), ldg,
                               st, 1, 0, 0, 0, 0, &pf, K_QR);
            }
        }
        // Ad <- Ad R^{-1} by recursive halving: Q_1 = A_1 R_11^{-1}, then
        // A_2 -= Q_1 R_12 on MFMA and Q_2 = A_2 R_22^{-1}; 64-column leaves by
        // row-wise substitution (backward stable, like the column-block order)
        trsm(0, r);
        // R accumulation: Rt = R_pass Rt
        if (!Rt) {
            Rt = (double2*)w.Z;
            launch_booked(pf, K_QR, 0.0, 32.0 * r * r, k_qr_triu, dim3((r + 255) / 256, r), dim3(256), 0, st,
                          (const double2*)w.G, ldg, r, Rt);
        } else {
            launch_booked(pf, K_QR, 0.0, 32.0 * r * r, k_qr_triu, dim3((r + 255) / 256, r), dim3(256), 0, st,
                          (const double2*)w.G, ldg, r, Rp);
            double2* Rn = Rt == (double2*)w.Z ? (double2*)w.U : (double2*)w.Z;
            zgemm<0, 0, 0>(r, r, r, Rp, r, Rt, r, Rn, r, st, 1, 0, 0, 0, 0, &pf, K_QR);
            Rt = Rn;
        }
    };
    auto failed = [&]() {
        if (hipMemcpyAsync(info_host, info, sizeof(DevInfo), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            throw HeevFailure{"Cholesky QR flag read"};
        return info_host->qr_fail != 0;
    };
    auto load = [&]() {
        launch_booked(pf, K_QR, 0.0, (double)m * r * (sizeof(C2<T>) + 16.0), k_to_f64<T>, dim3((m + 255) / 256, r),
                      dim3(256), 0, st, A, m, lda, Ad, ldx);
        Rt = nullptr;
    };
    load();
    pass_run(kQrPlain);
    pass_run(kQrFinal);
    if (failed()) {
        load();
        pass_run(kQrShifted);
        pass_run(kQrAfterShift);
        pass_run(kQrFinal);
        if (failed()) return false;
    }
    launch_booked(pf, K_QR, 0.0, (double)m * r * (16.0 + sizeof(C2<T>)), k_from_f64<T>, dim3((m + 255) / 256, r),
                  dim3(256), 0, st, (const double2*)Ad, ldx, m, Q, ldq);
    launch_booked(pf, K_QR, 0.0, (double)r * r * (16.0 + sizeof(C2<T>)), k_from_f64<T>, dim3((r + 255) / 256, r),
                  dim3(256), 0, st, (const double2*)Rt, r, r, R, r);
    if (hipGetLastError() != hipSuccess) throw HeevFailure{"Cholesky QR launch"};
    return true;
}

template bool cholqr3<double>(const double2*, int, int, int, double2*, int, double2*, DevInfo*, DevInfo*,
                              HeevWork&, Profiler&, hipStream_t);
template bool cholqr3<float>(const float2*, int, int, int, float2*, int, float2*, DevInfo*, DevInfo*, HeevWork&,
                             Profiler&, hipStream_t);

// Certificate of the eigen start: the largest relative off-diagonal of X^H X,
// measured in FP64 as the sweeps measure it, against tol.  Returns true when X
// is orthogonal to tol (then the sweeps can be skipped); reads the measure back
// through info_host (synchronises).
template <typename T>
bool heev_check(C2<T>* X, int m, int N, int ld, double tol, double zrel2, DevInfo* info, DevInfo* info_host,
                HeevWork& w, Profiler& pf, hipStream_t st) {
    const int ldx = ((w.cap_m + 1) & ~1) + 8;
    const int ldg = N + 8;
    launch_booked(pf, K_HGRAM, 0.0, (double)m * N * (sizeof(C2<T>) + 16.0), k_to_f64<T>, dim3((m + 255) / 256, N),
                  dim3(256), 0, st, (const C2<T>*)X, m, ld, w.Xd, ldx);
    zgemm<1, 0, 2>(N, N, m, w.Xd, ldx, w.Xd, ldx, w.G, ldg, st, 1, 0, 0, 0, 0, &pf, K_HGRAM);
    launch_booked(pf, K_HGRAM, 0.0, 24.0 * N, k_gram_diag, dim3(1), dim3(256), 0, st, (const double2*)w.G, ldg, N,
                  w.dv, info);
    launch_booked(pf, K_HGRAM, 0.0, 8.0 * (double)N * N, k_gram_offmax, dim3(4, N), dim3(256), 0, st,
                  (const double2*)w.G, ldg, N, zrel2, (const double*)w.dv, info);
    if (hipMemcpyAsync(info_host, info, sizeof(DevInfo), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        throw HeevFailure{"Gram check read"};
    double off;
    const unsigned long long bits = info_host->offmax_bits;
    std::memcpy(&off, &bits, sizeof(off));
    return off <= tol;
}

template bool heev_check<double>(double2*, int, int, int, double, double, DevInfo*, DevInfo*, HeevWork&,
                                 Profiler&, hipStream_t);
template bool heev_check<float>(float2*, int, int, int, double, double, DevInfo*, DevInfo*, HeevWork&,
                                Profiler&, hipStream_t);

}  // namespace mpo

// Complex GEMM on MFMA and the fused two-site contraction + channel kernel.
//
// theta = A_s . A_{s+1} (App. A, B^{[l,l+1]} before the map; "Note added":
// the two sites of the gate are contracted locally) and the 16x16 noisy-gate
// superoperator applied to each (a, c) pair of bond indices (App. A,
// definition of M acting on J_l J_{l+1}).
//
// Storage: site tensor A[a, I, c] at a + chiL*(I + 4*c) (column-major in both
// matricisations: L(A) = ((I,a) x c), R(A) = (a x (J,c))).  All matrices
// column-major.  A complex product costs 4 real MFMAs (re*re - im*im,
// re*im + im*re) accumulated into separate real and imaginary tiles.
#include "common.h"

namespace mpo {

constexpr int BM = 64, BN = 64, BK = 16;

// 64x64 output tile per 256-thread work-group; 4 waves in a 2x2 layout, each
// owning 32x32 = 2x2 MFMA tiles of 16x16.
template <typename T>
__device__ __forceinline__ void mma_tile(const C2<T> (*As)[BM + 1], const C2<T> (*Bs)[BN + 1],
                                         int lane, int wm, int wn, A4<T> (&accR)[2][2],
                                         A4<T> (&accI)[2][2]) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
        C2<T> a[2], b[2];
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
}

// The same 64x64 tile with split-BF16x3 products: one K = 16 step per call.
__device__ __forceinline__ void mma_tile_bf3(const float2 (*As)[BM + 1], const float2 (*Bs)[BN + 1],
                                             int lane, int wm, int wn, f4 (&accR)[2][2],
                                             f4 (&accI)[2][2]) {
    CBF a[2], b[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        float2 va[4], vb[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            va[j] = As[4 * (lane >> 4) + j][wm * 32 + q * 16 + (lane & 15)];
            vb[j] = Bs[4 * (lane >> 4) + j][wn * 32 + q * 16 + (lane & 15)];
        }
        a[q] = cbf_split(va, false);
        b[q] = cbf_split(vb, false);
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) cmfma_bf3(accR[bi][bj], accI[bi][bj], a[bi], b[bj]);
}

template <typename T, bool BF>
__device__ __forceinline__ void mma_step(const C2<T> (*As)[BM + 1], const C2<T> (*Bs)[BN + 1],
                                         int lane, int wm, int wn, A4<T> (&accR)[2][2],
                                         A4<T> (&accI)[2][2]) {
    if constexpr (BF) mma_tile_bf3(As, Bs, lane, wm, wn, accR, accI);
    else mma_tile<T>(As, Bs, lane, wm, wn, accR, accI);
}

// FP32 storage: the MFMA accumulators hold partial sums over at most kChunkK
// terms of K and are then added into FP64 sums.  One FP32 accumulator chain
// over the whole K (up to 4096 here) rounds once per 4 terms into a growing
// partial sum; for the cancelling sums of a re-gauge (rows of U^H A scale with
// the singular values) that rounding, relative to the result, grows with
// sigma_1 / sigma_k and was measured to dominate the FP32 mode's entropy error.
constexpr int kChunkK = 32;

__device__ __forceinline__ void flush_acc(f4 (&accR)[2][2], f4 (&accI)[2][2], d4 (&sumR)[2][2],
                                          d4 (&sumI)[2][2]) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                sumR[bi][bj][r] += (double)accR[bi][bj][r];
                sumI[bi][bj][r] += (double)accI[bi][bj][r];
                accR[bi][bj][r] = 0.f;
                accI[bi][bj][r] = 0.f;
            }
}

// Sum-side accumulator: FP64 for FP32 storage with FP32-MFMA products, none otherwise.
template <typename T, bool BF> struct SumAcc {
    static constexpr bool on = false;
    d4 R[1][1], I[1][1];
};
template <> struct SumAcc<float, false> {
    static constexpr bool on = true;
    d4 R[2][2], I[2][2];
};

template <typename T>
__device__ __forceinline__ void zero_acc(A4<T> (&accR)[2][2], A4<T> (&accI)[2][2]) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) { accR[bi][bj][r] = T(0); accI[bi][bj][r] = T(0); }
}

__device__ __forceinline__ void zero_sum(d4 (&sR)[2][2], d4 (&sI)[2][2]) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) { sR[bi][bj][r] = 0.0; sI[bi][bj][r] = 0.0; }
}

// C (M x N) = op(A) (M x K) * op(B) (K x N); op 0 = as stored, 1 = conj-transpose.
template <typename T, int OPA, int OPB, bool BF>
__global__ __launch_bounds__(256) void k_cgemm(int M, int N, int K, const C2<T>* __restrict__ A,
                                               int lda, const C2<T>* __restrict__ B, int ldb,
                                               C2<T>* __restrict__ Cm, int ldc) {
    __shared__ C2<T> As[BK][BM + 1];
    __shared__ C2<T> Bs[BK][BN + 1];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    A4<T> accR[2][2], accI[2][2];
    zero_acc<T>(accR, accI);
    SumAcc<T, BF> sum;
    if constexpr (SumAcc<T, BF>::on) zero_sum(sum.R, sum.I);
    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = t + 256 * r;
            int i, k;
            if (OPA == 0) { i = e & 63; k = e >> 6; } else { k = e & 15; i = e >> 4; }
            const int gi = m0 + i, gk = k0 + k;
            C2<T> v = czero<T>();
            if (gi < M && gk < K)
                v = (OPA == 0) ? A[gi + (size_t)gk * lda] : cconj<T>(A[gk + (size_t)gi * lda]);
            As[k][i] = v;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = t + 256 * r;
            int j, k;
            if (OPB == 0) { k = e & 15; j = e >> 4; } else { j = e & 63; k = e >> 6; }
            const int gj = n0 + j, gk = k0 + k;
            C2<T> v = czero<T>();
            if (gj < N && gk < K)
                v = (OPB == 0) ? B[gk + (size_t)gj * ldb] : cconj<T>(B[gj + (size_t)gk * ldb]);
            Bs[k][j] = v;
        }
        __syncthreads();
        mma_step<T, BF>(As, Bs, lane, wm, wn, accR, accI);
        __syncthreads();
        if constexpr (SumAcc<T, BF>::on)
            if ((k0 + BK) % kChunkK == 0 || k0 + BK >= K) flush_acc(accR, accI, sum.R, sum.I);
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = m0 + wm * 32 + bi * 16 + acc_row<T>(lane, r);
                const int j = n0 + wn * 32 + bj * 16 + (lane & 15);
                if (i < M && j < N) {
                    if constexpr (SumAcc<T, BF>::on)
                        Cm[i + (size_t)j * ldc] = cmake<T>((T)sum.R[bi][bj][r], (T)sum.I[bi][bj][r]);
                    else
                        Cm[i + (size_t)j * ldc] = cmake<T>(accR[bi][bj][r], accI[bi][bj][r]);
                }
            }
}

template <typename T, bool BF>
static void cgemm_dispatch(int opa, int opb, dim3 grid, int M, int N, int K, const C2<T>* A, int lda,
                           const C2<T>* B, int ldb, C2<T>* C, int ldc, hipStream_t st) {
    if (opa == 0 && opb == 0)
        hipLaunchKernelGGL((k_cgemm<T, 0, 0, BF>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc);
    else if (opa == 1 && opb == 0)
        hipLaunchKernelGGL((k_cgemm<T, 1, 0, BF>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc);
    else if (opa == 0 && opb == 1)
        hipLaunchKernelGGL((k_cgemm<T, 0, 1, BF>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc);
    else
        hipLaunchKernelGGL((k_cgemm<T, 1, 1, BF>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc);
}

template <typename T>
void launch_cgemm(int opa, int opb, int M, int N, int K, const C2<T>* A, int lda,
                  const C2<T>* B, int ldb, C2<T>* C, int ldc, hipStream_t st, bool bf3) {
    if (M <= 0 || N <= 0) return;
    dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN);
    if constexpr (sizeof(T) == 4) {
        if (bf3) { cgemm_dispatch<T, true>(opa, opb, grid, M, N, K, A, lda, B, ldb, C, ldc, st); return; }
    }
    cgemm_dispatch<T, false>(opa, opb, grid, M, N, K, A, lda, B, ldb, C, ldc, st);
}

// One work-group owns 16 left-bond values a and 16 right-bond values c, i.e.
// the 64 theta rows (I, a) and 64 columns (c, J) that the channel couples.
template <typename T, bool BF>
__global__ __launch_bounds__(256) void k_theta_channel(int chiL, int chiM, int chiR,
                                                       const C2<T>* __restrict__ As_g,
                                                       const C2<T>* __restrict__ Bs_g,
                                                       const C2<T>* __restrict__ Mdev,
                                                       C2<T>* __restrict__ X, C2<T>* __restrict__ X2,
                                                       int ldx) {
    __shared__ C2<T> Ms[16][16];
    __shared__ C2<T> As[BK][BM + 1];
    __shared__ C2<T> Bs[BK][BN + 1];
    __shared__ C2<T> Cs[64][65];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int a0 = blockIdx.x * 16, c0 = blockIdx.y * 16;
    const int m = 4 * chiL, K = chiM, ldb = chiM;
    Ms[t >> 4][t & 15] = Mdev[t];
    A4<T> accR[2][2], accI[2][2];
    zero_acc<T>(accR, accI);
    SumAcc<T, BF> sum;
    if constexpr (SumAcc<T, BF>::on) zero_sum(sum.R, sum.I);
    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = t + 256 * r;
            const int i = e & 63, k = e >> 6;
            const int a = a0 + (i & 15), I = i >> 4, gk = k0 + k;
            C2<T> v = czero<T>();
            if (a < chiL && gk < K) v = As_g[(a + chiL * I) + (size_t)gk * m];
            As[k][i] = v;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = t + 256 * r;
            const int k = e & 15, j = e >> 4;
            const int gcol = 4 * c0 + j, gk = k0 + k;
            C2<T> v = czero<T>();
            if (gcol < 4 * chiR && gk < K) v = Bs_g[gk + (size_t)gcol * ldb];
            Bs[k][j] = v;
        }
        __syncthreads();
        mma_step<T, BF>(As, Bs, lane, wm, wn, accR, accI);
        __syncthreads();
        if constexpr (SumAcc<T, BF>::on)
            if ((k0 + BK) % kChunkK == 0 || k0 + BK >= K) flush_acc(accR, accI, sum.R, sum.I);
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                C2<T> v;
                if constexpr (SumAcc<T, BF>::on) v = cmake<T>((T)sum.R[bi][bj][r], (T)sum.I[bi][bj][r]);
                else v = cmake<T>(accR[bi][bj][r], accI[bi][bj][r]);
                Cs[wm * 32 + bi * 16 + acc_row<T>(lane, r)][wn * 32 + bj * 16 + (lane & 15)] = v;
            }
    __syncthreads();
    const int al = t & 15, cl = t >> 4;
    const int a = a0 + al, c = c0 + cl;
    if (a < chiL && c < chiR) {
        C2<T> th[16];
#pragma unroll
        for (int ip = 0; ip < 4; ++ip)
#pragma unroll
            for (int jp = 0; jp < 4; ++jp) th[4 * ip + jp] = Cs[ip * 16 + al][cl * 4 + jp];
#pragma unroll
        for (int I = 0; I < 4; ++I)
#pragma unroll
            for (int J = 0; J < 4; ++J) {
                T re = T(0), im = T(0);
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const C2<T> mm = Ms[4 * I + J][q];
                    re += mm.x * th[q].x - mm.y * th[q].y;
                    im += mm.x * th[q].y + mm.y * th[q].x;
                }
                const size_t off = (size_t)(a + chiL * I) + (size_t)ldx * (J + 4 * c);
                X[off] = cmake<T>(re, im);
                if (X2) X2[off] = cmake<T>(re, im);
            }
    }
}

template <typename T>
void launch_theta_channel(int chiL, int chiM, int chiR, const C2<T>* As, const C2<T>* Bs,
                          const C2<T>* Mdev, C2<T>* X, C2<T>* X2, int ldx, hipStream_t st, bool bf3) {
    dim3 grid((chiL + 15) / 16, (chiR + 15) / 16);
    if constexpr (sizeof(T) == 4) {
        if (bf3) {
            hipLaunchKernelGGL((k_theta_channel<T, true>), grid, dim3(256), 0, st, chiL, chiM, chiR,
                               As, Bs, Mdev, X, X2, ldx);
            return;
        }
    }
    hipLaunchKernelGGL((k_theta_channel<T, false>), grid, dim3(256), 0, st, chiL, chiM, chiR, As, Bs,
                       Mdev, X, X2, ldx);
}

template void launch_cgemm<double>(int, int, int, int, int, const double2*, int, const double2*,
                                   int, double2*, int, hipStream_t, bool);
template void launch_cgemm<float>(int, int, int, int, int, const float2*, int, const float2*, int,
                                  float2*, int, hipStream_t, bool);
template void launch_theta_channel<double>(int, int, int, const double2*, const double2*,
                                           const double2*, double2*, double2*, int, hipStream_t, bool);
template void launch_theta_channel<float>(int, int, int, const float2*, const float2*,
                                          const float2*, float2*, float2*, int, hipStream_t, bool);

}  // namespace mpo

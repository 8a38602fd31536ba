// Blocked one-sided Jacobi SVD for the truncated split (App. A: SVD of the
// two-site block, keep the largest singular values).
//
// The columns of X (m x N, column-major) are orthogonalised by right-
// multiplication with unitary matrices: blocks of 32 columns are paired in a
// round-robin tournament; for a pair the 64x64 Gram matrix is formed on MFMA,
// diagonalised by a cyclic two-sided Jacobi sweep in FP64 inside one
// work-group, and the resulting 64x64 unitary is applied to the pair's
// columns on MFMA.  At convergence X V = U Sigma with orthogonal columns, so
// the left singular vectors are the normalised columns and the singular
// values their norms.  Columns are re-ordered by decreasing norm before each
// sweep through an index map (no data movement).
#include <hip/hip_ext.h>

#include "common.h"
#include <cstdio>
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>

namespace mpo {

// Block sizes: JB columns per block, 2*JB per pair (JB = 16 or 32).

// Round-robin tournament (circle method) over nb players (nb even):
// pair 0 of round r is (r, nb-1); pair i > 0 is (r+i, r-i) mod (nb-1).
__host__ __device__ __forceinline__ void pair_of(int round, int i, int nb, int& p, int& q) {
    const int M = nb - 1;
    if (i == 0) { p = round; q = M; }
    else { p = (round + i) % M; q = (round - i + M) % M; }
}

// ------------------------------------------------------------- column norms
template <typename T>
__global__ __launch_bounds__(256) void k_colnorm2(const C2<T>* __restrict__ X, int m, int N, int ld,
                                                  double* __restrict__ out, const int* __restrict__ halt) {
    if (halt && *halt) return;
    const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (col >= N) return;
    const C2<T>* x = X + (size_t)col * ld;
    double s = 0.0;
    for (int i = lane; i < m; i += 64) {
        const double2 v = to_d2(x[i]);
        s += v.x * v.x + v.y * v.y;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) out[col] = s;
}

// ------------------------------------------- sort by decreasing norm (bitonic)
// Ties keep ascending column index, so the order is deterministic.
__global__ __launch_bounds__(1024) void k_sort_desc(const double* __restrict__ nrm2, int N,
                                                    int* __restrict__ colmap,
                                                    double* __restrict__ sig2,
                                                    double* __restrict__ fro2,
                                                    const int* __restrict__ halt) {
    if (halt && *halt) return;
    __shared__ double key[4096];
    __shared__ int idx[4096];
    __shared__ double red[1024];
    const int t = threadIdx.x;
    int P2 = 1;
    while (P2 < N) P2 <<= 1;
    double part = 0.0;
    for (int e = t; e < P2; e += 1024) {
        const double v = e < N ? nrm2[e] : -1.0;
        key[e] = v;
        idx[e] = e;
        if (e < N) part += v;
    }
    red[t] = part;
    __syncthreads();
    for (int k = 2; k <= P2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int e = t; e < P2; e += 1024) {
                const int f = e ^ j;
                if (f > e) {
                    const double ke = key[e], kf = key[f];
                    const int ie = idx[e], jf = idx[f];
                    const bool e_less = (ke < kf) || (ke == kf && ie > jf);
                    const bool f_less = (kf < ke) || (kf == ke && jf > ie);
                    const bool swap = ((e & k) == 0) ? e_less : f_less;
                    if (swap) { key[e] = kf; key[f] = ke; idx[e] = jf; idx[f] = ie; }
                }
            }
            __syncthreads();
        }
    }
    for (int e = t; e < N; e += 1024) { colmap[e] = idx[e]; sig2[e] = key[e]; }
    for (int o = 512; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    if (t == 0 && fro2) *fro2 = red[0];
}

// ------------------------------------------------------------- pair Gram
// partials[(pair*splits + split)*NB*NB + i + NB*j] = sum_rows conj(x_i) x_j over
// this split's row range, for the NB = 2*JB columns of the pair, in FP64.  The
// Gram matrix is Hermitian, so only its upper 16x16 tiles are computed (TB
// column tiles loaded once per step feed TB(TB+1)/2 complex MFMA products) and
// the lower ones are written as conjugates.  Each wave sums its products in the
// working precision over a few dozen rows, then in FP64; the four waves of a
// work-group are added in LDS.  One kernel per mode, each the fastest measured
// on gfx950 for its operand size.

// Adds the four waves' FP64 tile sums and writes the pair's NB x NB partial.
template <typename T, int NB>
__device__ __forceinline__ void gram_finish(const d4* sumR, const d4* sumI, double2* red,
                                            double2* __restrict__ out) {
    constexpr int TB = NB / 16, NU = TB * (TB + 1) / 2;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int u = 0; u < NU; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int idx = u * 256 + acc_row<T>(lane, r) + 16 * (lane & 15);
                    if (w == 0) red[idx] = make_double2(sumR[u][r], sumI[u][r]);
                    else { red[idx].x += sumR[u][r]; red[idx].y += sumI[u][r]; }
                }
        }
        __syncthreads();
    }
    for (int e = t; e < NB * NB; e += 256) {
        const int i = e % NB, j = e / NB;
        const int bi = i >> 4, bj = j >> 4;
        double2 v;
        if (bi <= bj) {
            const int u = bi * TB - bi * (bi - 1) / 2 + (bj - bi);
            v = red[u * 256 + (i & 15) + 16 * (j & 15)];
        } else {
            const int u = bj * TB - bj * (bj - 1) / 2 + (bi - bj);
            const double2 w = red[u * 256 + (j & 15) + 16 * (i & 15)];
            v = make_double2(w.x, -w.y);
        }
        out[i + NB * j] = v;
    }
}

// Split-BF16x3 mode: 128-row slabs are staged in LDS by the whole work-group
// (the next slab is loaded into registers while the current one is reduced);
// each wave takes a quarter of every slab, 16 rows per step through
// v_mfma_f32_16x16x16_bf16 with hi/lo operands.
template <int JB>
__global__ __launch_bounds__(256) void k_pair_gram_bf3(const float2* __restrict__ X, int m, int N, int ld,
                                                       const int* __restrict__ colmap, int nb,
                                                       int round, int splits, int chunk,
                                                       double2* __restrict__ partials,
                                 const int* __restrict__ halt) {
    if (*halt) return;
    using T = float;
    constexpr int NB = 2 * JB, TB = NB / 16, NU = TB * (TB + 1) / 2;
    constexpr int RB = 4096 / NB;              // rows per staged slab
    constexpr int RW = RB / 4;                 // rows of a slab per wave
    __shared__ C2<T> Xs[RB][NB + 1];
    __shared__ double2 red[NU * 256];
    __shared__ int cols[NB];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int pair = blockIdx.x, split = blockIdx.y;
    int p, q;
    pair_of(round, pair, nb, p, q);
    if (t < NB) {
        const int lj = (t < JB) ? p * JB + t : q * JB + (t - JB);
        cols[t] = (lj < N) ? colmap[lj] : -1;
    }
    __syncthreads();
    const int r0 = split * chunk;
    const int r1 = min(m, r0 + chunk);
    A4<T> accR[NU], accI[NU];
    d4 sumR[NU], sumI[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) { sumR[u][r] = 0.0; sumI[u][r] = 0.0; }
    // the next slab is loaded into registers while the current one is reduced
    constexpr int LE = (RB * NB) / 256;        // slab elements per thread
    C2<T> pre[LE];
#pragma unroll
    for (int r = 0; r < LE; ++r) {
        const int e = t + 256 * r;
        const int row = e % RB, c = cols[e / RB];
        pre[r] = (c >= 0 && r0 + row < r1) ? X[(size_t)(r0 + row) + (size_t)ld * c] : czero<T>();
    }
    for (int k0 = r0; k0 < r1; k0 += RB) {
#pragma unroll
        for (int r = 0; r < LE; ++r) {
            const int e = t + 256 * r;
            Xs[e % RB][e / RB] = pre[r];
        }
        __syncthreads();
        if (k0 + RB < r1) {
            const int k1 = k0 + RB;
#pragma unroll
            for (int r = 0; r < LE; ++r) {
                const int e = t + 256 * r;
                const int row = e % RB, c = cols[e / RB];
                pre[r] = (c >= 0 && k1 + row < r1) ? X[(size_t)(k1 + row) + (size_t)ld * c] : czero<T>();
            }
        }
#pragma unroll
        for (int u = 0; u < NU; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) { accR[u][r] = T(0); accI[u][r] = T(0); }
        {
            for (int kk = wave * RW; kk < (wave + 1) * RW; kk += 16) {
                const bf4 sign = {(short)0x8000, (short)0x8000, (short)0x8000, (short)0x8000};
                CBF xb[TB], xa[TB];        // x and conj(x), rows kk + 4(l/16) + j
#pragma unroll
                for (int b = 0; b < TB; ++b) {
                    float2 v[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) v[j] = Xs[kk + 4 * (lane >> 4) + j][b * 16 + (lane & 15)];
                    xb[b] = cbf_split(v, false);
                    xa[b] = xb[b];
                    xa[b].ih = xb[b].ih ^ sign;
                    xa[b].il = xb[b].il ^ sign;
                }
                int u = 0;
#pragma unroll
                for (int bi = 0; bi < TB; ++bi)
#pragma unroll
                    for (int bj = bi; bj < TB; ++bj, ++u) cmfma_bf3(accR[u], accI[u], xa[bi], xb[bj]);
            }
        }
#pragma unroll
        for (int u = 0; u < NU; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                sumR[u][r] += (double)accR[u][r];
                sumI[u][r] += (double)accI[u][r];
            }
        __syncthreads();
    }
    gram_finish<T, NB>(sumR, sumI, red, partials + (size_t)(pair * splits + split) * (NB * NB));
}

// FP64 mode: every wave works through its own rows with no work-group barrier
// in the main loop; wave w takes rows [s, s + WR) of every 4*WR-row slab of the
// split's range.  A slab (NB columns x WR rows, 8 KiB) is read with coalesced
// 16-byte loads, 16 lanes covering 256 contiguous bytes of one column, and
// transposed through a wave-private LDS buffer (column pitch 17 x 16 bytes, so
// that both the stores and the 16-byte operand reads meet the minimum bank
// multiplicity) into MFMA operand layout.  The rows of a dot product may be
// summed in any order as long as both operands follow it: lane (i, k) takes 16
// contiguous bytes of column i (one FP64 row, two FP32 rows) as its k-th
// operand.  The next slab's loads are in flight while the current one is
// multiplied.
// 16 bytes of one column: two FP32 rows or one FP64 row (Gram and update loads)
template <typename T> struct GramLoad;
template <> struct GramLoad<float> { using type = float4; };     // re, im of rows r, r+1
template <> struct GramLoad<double> { using type = double2; };   // re, im of row r

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, int JB>
__global__ __launch_bounds__(256) void k_pair_gram_lds(const C2<T>* __restrict__ X, int m, int N, int ld,
                                                       const int* __restrict__ colmap, int nb,
                                                       int round, int splits, int chunk,
                                                       double2* __restrict__ partials,
                                 const int* __restrict__ halt) {
    if (*halt) return;
    constexpr int NB = 2 * JB, TB = NB / 16, NU = TB * (TB + 1) / 2;
    constexpr int E = 16 / (int)sizeof(C2<T>);   // rows per 16-byte unit
    constexpr int NS = 4;                         // MFMA k-steps per slab
    constexpr int WR = NS * 4 * E;                // rows per wave and slab (16 units)
    constexpr int NI = NB / 4;                    // 16-byte loads per lane and slab
    constexpr int PW = 17;                        // column pitch in 16-byte units
    using LV = typename GramLoad<T>::type;
    __shared__ LV slab[4][NB * PW];
    __shared__ double2 red[NU * 256];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int pair = blockIdx.x, split = blockIdx.y;
    int p, q;
    pair_of(round, pair, nb, p, q);
    // load layout: lane l reads unit (l & 15) of column 4j + (l >> 4) in load j
    const int lu = lane & 15;
    const C2<T>* colp[NI];
    bool live[NI];
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        const int c = 4 * j + (lane >> 4);
        const int lj = c < JB ? p * JB + c : q * JB + (c - JB);
        const int col = lj < N ? colmap[lj] : -1;
        live[j] = col >= 0;
        colp[j] = X + (size_t)ld * (live[j] ? col : 0);
    }
    const int r0 = split * chunk;
    const int r1 = min(m, r0 + chunk);
    const bool aligned = (ld % E) == 0;           // 16-byte loads need an even column stride in FP32
    auto load = [&](int j, int row) -> LV {
        if constexpr (E == 2) {
            if (live[j] && aligned && row + 1 < r1) return *reinterpret_cast<const float4*>(colp[j] + row);
            const float2 a = (live[j] && row < r1) ? colp[j][row] : make_float2(0.f, 0.f);
            const float2 c = (live[j] && row + 1 < r1) ? colp[j][row + 1] : make_float2(0.f, 0.f);
            return make_float4(a.x, a.y, c.x, c.y);
        } else {
            return (live[j] && row < r1) ? colp[j][row] : make_double2(0.0, 0.0);
        }
    };
    LV* ls = slab[wave];
    const int ci = lane & 15, kq = lane >> 4;
    A4<T> accR[NU], accI[NU];
    d4 sumR[NU], sumI[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) { sumR[u][r] = 0.0; sumI[u][r] = 0.0; }
    LV nxt[NI];
    int s = r0 + wave * WR;
    if (s < r1) {
#pragma unroll
        for (int j = 0; j < NI; ++j) nxt[j] = load(j, s + lu * E);
    }
    for (; s < r1; s += 4 * WR) {
#pragma unroll
        for (int j = 0; j < NI; ++j) ls[(4 * j + (lane >> 4)) * PW + lu] = nxt[j];
        wave_sync();
        const int sn = s + 4 * WR;
        if (sn < r1) {
#pragma unroll
            for (int j = 0; j < NI; ++j) nxt[j] = load(j, sn + lu * E);
        }
#pragma unroll
        for (int u = 0; u < NU; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) { accR[u][r] = T(0); accI[u][r] = T(0); }
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            LV v[TB];
#pragma unroll
            for (int b = 0; b < TB; ++b) v[b] = ls[(b * 16 + ci) * PW + 4 * st + kq];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                T xr[TB], xi[TB];
#pragma unroll
                for (int b = 0; b < TB; ++b) {
                    if constexpr (E == 2) {
                        xr[b] = e == 0 ? v[b].x : v[b].z;
                        xi[b] = e == 0 ? v[b].y : v[b].w;
                    } else {
                        xr[b] = v[b].x;
                        xi[b] = v[b].y;
                    }
                }
                int u = 0;
#pragma unroll
                for (int bi = 0; bi < TB; ++bi)
#pragma unroll
                    for (int bj = bi; bj < TB; ++bj, ++u) {
                        // conj(x_bi) x_bj: (ar - i ai)(br + i bi)
                        accR[u] = mfma16(xr[bi], xr[bj], accR[u]);
                        accR[u] = mfma16(xi[bi], xi[bj], accR[u]);
                        accI[u] = mfma16(xr[bi], xi[bj], accI[u]);
                        accI[u] = mfma16(-xi[bi], xr[bj], accI[u]);
                    }
            }
        }
        wave_sync();   // the slab buffer is rewritten next
#pragma unroll
        for (int u = 0; u < NU; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                sumR[u][r] += (double)accR[u][r];
                sumI[u][r] += (double)accI[u][r];
            }
    }
    gram_finish<T, NB>(sumR, sumI, red, partials + (size_t)(pair * splits + split) * (NB * NB));
}

// FP32 mode: as in the FP64 kernel, but lane (i, k) loads its 16 bytes of
// column i straight into operand registers (16 columns x 64 bytes per load),
// with no LDS in the main loop.  The loads are less regular than the LDS
// kernel's (the 16 columns of a load share L1 sets when m is a power of two),
// but on gfx950 this measured faster for FP32, whose slab carries half the MFMA
// work of an FP64 one; for FP64 the LDS kernel is faster.
template <typename T, int JB>
__global__ __launch_bounds__(256) void k_pair_gram_regs(const C2<T>* __restrict__ X, int m, int N, int ld,
                                                        const int* __restrict__ colmap, int nb,
                                                        int round, int splits, int chunk,
                                                        double2* __restrict__ partials,
                                 const int* __restrict__ halt) {
    if (*halt) return;
    constexpr int NB = 2 * JB, TB = NB / 16, NU = TB * (TB + 1) / 2;
    constexpr int E = 16 / (int)sizeof(C2<T>);
    constexpr int NS = 4;
    constexpr int WR = NS * 4 * E;
    using LV = typename GramLoad<T>::type;
    __shared__ double2 red[NU * 256];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int ci = lane & 15, kq = lane >> 4;
    const int pair = blockIdx.x, split = blockIdx.y;
    int p, q;
    pair_of(round, pair, nb, p, q);
    const C2<T>* colp[TB];
    bool live[TB];
#pragma unroll
    for (int b = 0; b < TB; ++b) {
        const int c = b * 16 + ci;
        const int lj = c < JB ? p * JB + c : q * JB + (c - JB);
        const int col = lj < N ? colmap[lj] : -1;
        live[b] = col >= 0;
        colp[b] = X + (size_t)ld * (live[b] ? col : 0);
    }
    const int r0 = split * chunk;
    const int r1 = min(m, r0 + chunk);
    const bool aligned = (ld % E) == 0;
    auto load = [&](int b, int row) -> LV {
        if constexpr (E == 2) {
            if (live[b] && aligned && row + 1 < r1) return *reinterpret_cast<const float4*>(colp[b] + row);
            const float2 a = (live[b] && row < r1) ? colp[b][row] : make_float2(0.f, 0.f);
            const float2 c = (live[b] && row + 1 < r1) ? colp[b][row + 1] : make_float2(0.f, 0.f);
            return make_float4(a.x, a.y, c.x, c.y);
        } else {
            return (live[b] && row < r1) ? colp[b][row] : make_double2(0.0, 0.0);
        }
    };
    A4<T> accR[NU], accI[NU];
    d4 sumR[NU], sumI[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) { sumR[u][r] = 0.0; sumI[u][r] = 0.0; }
    LV cur[TB][NS], nxt[TB][NS];
    int s = r0 + wave * WR;
    if (s < r1) {
#pragma unroll
        for (int st = 0; st < NS; ++st)
#pragma unroll
            for (int b = 0; b < TB; ++b) cur[b][st] = load(b, s + st * 4 * E + kq * E);
    }
    for (; s < r1; s += 4 * WR) {
        const int sn = s + 4 * WR;
        if (sn < r1) {
#pragma unroll
            for (int st = 0; st < NS; ++st)
#pragma unroll
                for (int b = 0; b < TB; ++b) nxt[b][st] = load(b, sn + st * 4 * E + kq * E);
        }
#pragma unroll
        for (int u = 0; u < NU; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) { accR[u][r] = T(0); accI[u][r] = T(0); }
#pragma unroll
        for (int st = 0; st < NS; ++st)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                T xr[TB], xi[TB];
#pragma unroll
                for (int b = 0; b < TB; ++b) {
                    if constexpr (E == 2) {
                        xr[b] = e == 0 ? cur[b][st].x : cur[b][st].z;
                        xi[b] = e == 0 ? cur[b][st].y : cur[b][st].w;
                    } else {
                        xr[b] = cur[b][st].x;
                        xi[b] = cur[b][st].y;
                    }
                }
                int u = 0;
#pragma unroll
                for (int bi = 0; bi < TB; ++bi)
#pragma unroll
                    for (int bj = bi; bj < TB; ++bj, ++u) {
                        accR[u] = mfma16(xr[bi], xr[bj], accR[u]);
                        accR[u] = mfma16(xi[bi], xi[bj], accR[u]);
                        accI[u] = mfma16(xr[bi], xi[bj], accI[u]);
                        accI[u] = mfma16(-xi[bi], xr[bj], accI[u]);
                    }
            }
#pragma unroll
        for (int u = 0; u < NU; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                sumR[u][r] += (double)accR[u][r];
                sumI[u][r] += (double)accI[u][r];
            }
#pragma unroll
        for (int st = 0; st < NS; ++st)
#pragma unroll
            for (int b = 0; b < TB; ++b) cur[b][st] = nxt[b][st];
    }
    gram_finish<T, NB>(sumR, sumI, red, partials + (size_t)(pair * splits + split) * (NB * NB));
}

// --------------------------------------------------- NB x NB Hermitian eigen (FP64)
// Sums the Gram partials, measures the largest relative off-diagonal element
// |g_ij| / sqrt(g_ii g_jj), and if it exceeds tol runs up to inner_max cyclic
// Jacobi sweeps (parallel ordering: NB/2 disjoint rotations per step), giving
// a unitary W with W^H G W close to diagonal.  In a step every thread owns
// 2x2 blocks G[{i1,j1}][{i2,j2}], computes the two rotations it needs itself
// and applies G <- J1^H G J2 to its blocks (rows and columns at once) and J1
// to the matching entries of W; inactive pairs use the exact identity.
// Columns whose squared norm is at most zrel2 * ||X||_F^2 are never rotated.
__device__ __forceinline__ double2 dmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 dmulc(double2 a, double2 b) {   // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// 1/sqrt(x) for normal x > 0: hardware estimate and two Newton steps, each
// y <- y + y (1 - x y^2) / 2, which take it to full FP64 accuracy.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double e = fma(-x * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

// Rotation J = [[c, s], [-conj(s), c]] (c real, c^2 + |s|^2 = 1) with
// (J^H B J)_{01} = 0 for B = [[a, g], [conj(g), d]], through the smaller
// angle: with h = d - a and r = sqrt(h^2 + 4|g|^2), c^2 = (1 + |h|/r)/2 and
// s = sign(h) g / (r c).  Every term is a sum of non-negative parts, so small
// angles keep full relative accuracy.  The identity is returned when either
// column is at the rounding floor (squared norm <= zthr) or the pair is
// already orthogonal to tol.  The code has no branches, so the two rotations
// a thread needs are computed side by side; every thread that needs a pair's
// rotation computes it from the same values with the same operations, so all
// of them agree bit for bit.
__device__ __forceinline__ void pair_rotation(double a, double d, double2 g, double zthr,
                                              double tol2, double& c, double2& s) {
    const double g2 = fma(g.x, g.x, g.y * g.y);
    const bool act = (a > zthr) & (d > zthr) & (g2 > tol2 * a * d);
    const double h = d - a;
    const double inv_r = rsqrt_nr(act ? fma(h, h, 4.0 * g2) : 1.0);
    const double c2 = act ? fma(0.5 * fabs(h), inv_r, 0.5) : 1.0;
    const double inv_c = rsqrt_nr(c2);
    const double f = act ? (h >= 0.0 ? inv_r : -inv_r) * inv_c : 0.0;
    c = act ? c2 * inv_c : 1.0;
    s = make_double2(f * g.x, f * g.y);
}

// The same rotation from the hardware reciprocal square root estimate alone
// (relative error below 2^-24), made unitary to FP64 rounding afterwards:
// with e = c~^2 + |s~|^2 - 1 (about 2^-22), (c, s) = (c~, s~)(1 - e/2 + 3e^2/8)
// leaves c^2 + |s|^2 - 1 of order e^3.  The angle is off by about 2^-23, so
// the pair keeps an off-diagonal of that relative size, far below the outer
// tolerance of the FP32 and BF16x3 modes; the dependent chain is 14 operations
// instead of 21.
__device__ __forceinline__ void pair_rotation_fast(double a, double d, double2 g, double zthr,
                                                   double tol2, double& c, double2& s) {
    const double g2 = fma(g.x, g.x, g.y * g.y);
    const bool act = (a > zthr) & (d > zthr) & (g2 > tol2 * a * d);
    const double h = d - a;
    const double inv_r = __builtin_amdgcn_rsq(act ? fma(h, h, 4.0 * g2) : 1.0);
    const double c2 = act ? fma(0.5 * fabs(h), inv_r, 0.5) : 1.0;
    const double inv_c = __builtin_amdgcn_rsq(c2);
    const double ct = c2 * inv_c;
    const double f = act ? (h >= 0.0 ? inv_r : -inv_r) * inv_c : 0.0;
    const double sx = f * g.x, sy = f * g.y;
    const double e = fma(sy, sy, fma(sx, sx, fma(ct, ct, -1.0)));
    const double k = fma(e, fma(e, 0.375, -0.5), 1.0);
    c = act ? ct * k : 1.0;
    s = make_double2(sx * k, sy * k);
}

// Largest relative off-diagonal |g_ij| / sqrt(g_ii g_jj) over the columns
// above the rounding floor, and the set of round-robin steps (bit s) that pair
// at least one (i, j) above tol.  Pair (i, j), i, j < NB-1, meets at the step
// s with i + j = 2s (mod NB-1); the fixed member NB-1 meets i at step i.
template <int NB, int NT>
__device__ double block_scan(const double2 (*G)[NB + 2], double zthr, double tol2, double* red,
                             unsigned long long* smask, unsigned long long& mask) {
    constexpr int M = NB - 1;
    const int t = threadIdx.x;
    if (t == 0) *smask = 0ull;
    __syncthreads();
    double mx = 0.0;
    unsigned long long bits = 0ull;
    for (int e = t; e < NB * NB; e += NT) {
        const int i = e % NB, j = e / NB;
        if (i < j) {
            const double a = G[i][i].x, d = G[j][j].x;
            if (a > zthr && d > zthr) {
                const double2 g = G[i][j];
                const double g2 = fma(g.x, g.x, g.y * g.y);
                mx = fmax(mx, sqrt(g2) / sqrt(a * d));
                if (g2 > tol2 * a * d) {
                    const int st = (j == M) ? i : ((i + j) * ((M + 1) / 2)) % M;
                    bits |= 1ull << st;
                }
            }
        }
    }
    red[t] = mx;
    if (bits) atomicOr(smask, bits);
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
        if (t < o) red[t] = fmax(red[t], red[t + o]);
        __syncthreads();
    }
    const double r = red[0];
    mask = *smask;
    __syncthreads();
    return r;
}

constexpr int kEigThreads = 512;   // waves 0-3 transform G, waves 4-7 accumulate W

template <typename T, int JB>
__global__ __launch_bounds__(kEigThreads) void k_pair_eig(const double2* __restrict__ partials,
                                                         int splits, double tol, double zrel2,
                                                         const double* __restrict__ fro2,
                                                         int inner_max, C2<T>* __restrict__ Wout,
                                                         int* __restrict__ skip, DevInfo* info) {
    if (info->done) return;
    constexpr int NT = kEigThreads, NB = 2 * JB, NP = JB, U = NP * NP / 256;   // blocks per thread
    static_assert(NP * NP % 256 == 0, "block count must fill four waves");
    // Row pitch NB + 2 for G: the pair entries G[s+P][s-P] of one step then
    // fall in distinct banks (pitch NB + 1 maps them all to one bank).
    __shared__ double2 G[NB][NB + 2];
    __shared__ double2 W[NB][NB + 1];
    __shared__ double red[NT];
    __shared__ double rc[2][NP];       // rotations of the last two steps, for the W waves
    __shared__ double2 rs[2][NP];
    __shared__ unsigned long long smask;
    const int t = threadIdx.x, pair = blockIdx.x;
    for (int e = t; e < NB * NB; e += NT) {
        const int i = e % NB, j = e / NB;
        double2 s = make_double2(0.0, 0.0);
#pragma unroll 4
        for (int sp = 0; sp < splits; ++sp) {
            const double2 v = partials[(size_t)(pair * splits + sp) * (NB * NB) + i + NB * j];
            s.x += v.x;
            s.y += v.y;
        }
        G[i][j] = s;
    }
    __syncthreads();
    for (int e = t; e < NB * NB; e += NT) {
        const int i = e % NB, j = e / NB;
        if (i < j) {
            const double2 a = G[i][j], b = G[j][i];
            const double2 h = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
            G[i][j] = h;
            G[j][i] = make_double2(h.x, -h.y);
        } else if (i == j) {
            G[i][i].y = 0.0;
        }
    }
    __syncthreads();
    const double zthr = zrel2 * (*fro2);
    const double tol2 = tol * tol;
    unsigned long long mask;
    const double off0 = block_scan<NB, NT>(G, zthr, tol2, red, &smask, mask);
    if (off0 <= tol) {
        if (t == 0) skip[pair] = 1;
        return;
    }
    for (int e = t; e < NB * NB; e += NT) {
        const int i = e % NB, j = e / NB;
        W[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    // Thread tt of either half owns the 2x2 blocks b = tt + 256u, (P1, P2) =
    // (b / NP, b % NP).  A G thread rebuilds the rotations of P1 and P2 from
    // the diagonal blocks of G (all of them are read before any is
    // overwritten) and applies G <- J1^H G J2 to its block; the rotations of
    // the step are published for the W threads, which apply W <- W J1 to rows
    // {i2, j2} one step later, off the critical path of G.  A sweep visits
    // only the steps that held an entry above tol when it started (threshold
    // Jacobi: every other rotation of such a step is the identity).
    const bool gthr = t < 256;
    const int tt = t & 255;
    int steps_done = 0, k = 0, prev = 0;   // k counts executed steps, prev is the last one
    for (int sweep = 0; sweep < inner_max; ++sweep) {
        for (; mask; mask &= mask - 1, ++k) {
            const int step = __ffsll((long long)mask) - 1;
            ++steps_done;
            int i1[U], j1[U], i2[U], j2[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int b = tt + 256 * u;
                const int sp = gthr ? step : prev;   // W threads work on the previous step
                pair_of(sp, b / NP, NB, i1[u], j1[u]);
                pair_of(sp, b % NP, NB, i2[u], j2[u]);
            }
            double2 bk[U][4], s1[U], s2[U];
            double c1[U], c2[U];
            if (gthr) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    bk[u][0] = G[i1[u]][i2[u]];
                    bk[u][1] = G[i1[u]][j2[u]];
                    bk[u][2] = G[j1[u]][i2[u]];
                    bk[u][3] = G[j1[u]][j2[u]];
                    if constexpr (sizeof(T) == 8) {   // exact angles for the FP64 mode
                        pair_rotation(G[i2[u]][i2[u]].x, G[j2[u]][j2[u]].x, G[i2[u]][j2[u]], zthr,
                                      tol2, c2[u], s2[u]);
                    } else {
                        pair_rotation_fast(G[i2[u]][i2[u]].x, G[j2[u]][j2[u]].x, G[i2[u]][j2[u]],
                                           zthr, tol2, c2[u], s2[u]);
                    }
                    if constexpr (U == 1) {
                        // lane q < 16 of this wave holds rotation q as its P2 rotation, and
                        // P1 = 4 * wave + lane / 16 < 16: fetch it instead of recomputing
                        const int src = 4 * (tt >> 6) + ((tt & 63) >> 4);
                        c1[u] = __shfl(c2[u], src);
                        s1[u] = make_double2(__shfl(s2[u].x, src), __shfl(s2[u].y, src));
                    } else if constexpr (sizeof(T) == 8) {
                        pair_rotation(G[i1[u]][i1[u]].x, G[j1[u]][j1[u]].x, G[i1[u]][j1[u]], zthr,
                                      tol2, c1[u], s1[u]);
                    } else {
                        pair_rotation_fast(G[i1[u]][i1[u]].x, G[j1[u]][j1[u]].x, G[i1[u]][j1[u]],
                                           zthr, tol2, c1[u], s1[u]);
                    }
                }
                if (tt < NP) {          // P1 == 0: publish rotation P2 = tt
                    rc[k & 1][tt] = c2[0];
                    rs[k & 1][tt] = s2[0];
                }
            } else if (k > 0) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int P1 = (tt + 256 * u) / NP;
                    c1[u] = rc[(k - 1) & 1][P1];
                    s1[u] = rs[(k - 1) & 1][P1];
                    bk[u][0] = W[i2[u]][i1[u]];
                    bk[u][1] = W[i2[u]][j1[u]];
                    bk[u][2] = W[j2[u]][i1[u]];
                    bk[u][3] = W[j2[u]][j1[u]];
                }
            }
            __syncthreads();
            if (gthr) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const double2 b00 = bk[u][0], b01 = bk[u][1], b10 = bk[u][2], b11 = bk[u][3];
                    const double c1u = c1[u], c2u = c2[u];
                    // C = B J2: column i2 <- c2 B_i2 - conj(s2) B_j2, column j2 <- s2 B_i2 + c2 B_j2
                    const double2 t01 = dmulc(s2[u], b01), t11 = dmulc(s2[u], b11);
                    const double2 u00 = dmul(s2[u], b00), u10 = dmul(s2[u], b10);
                    const double2 c00 = make_double2(c2u * b00.x - t01.x, c2u * b00.y - t01.y);
                    const double2 c10 = make_double2(c2u * b10.x - t11.x, c2u * b10.y - t11.y);
                    const double2 c01 = make_double2(u00.x + c2u * b01.x, u00.y + c2u * b01.y);
                    const double2 c11 = make_double2(u10.x + c2u * b11.x, u10.y + c2u * b11.y);
                    // D = J1^H C: row i1 <- c1 C_i1 - s1 C_j1, row j1 <- conj(s1) C_i1 + c1 C_j1
                    const double2 v10 = dmul(s1[u], c10), v11 = dmul(s1[u], c11);
                    const double2 x00 = dmulc(s1[u], c00), x01 = dmulc(s1[u], c01);
                    G[i1[u]][i2[u]] = make_double2(c1u * c00.x - v10.x, c1u * c00.y - v10.y);
                    G[i1[u]][j2[u]] = make_double2(c1u * c01.x - v11.x, c1u * c01.y - v11.y);
                    G[j1[u]][i2[u]] = make_double2(x00.x + c1u * c10.x, x00.y + c1u * c10.y);
                    G[j1[u]][j2[u]] = make_double2(x01.x + c1u * c11.x, x01.y + c1u * c11.y);
                }
            } else if (k > 0) {
                // W <- W J1 on rows i2, j2 with the previous step's pairing
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const double2 w00 = bk[u][0], w01 = bk[u][1], w10 = bk[u][2], w11 = bk[u][3];
                    const double c1u = c1[u];
                    const double2 q0 = dmulc(s1[u], w01), q1 = dmulc(s1[u], w11);
                    const double2 r0 = dmul(s1[u], w00), r1 = dmul(s1[u], w10);
                    W[i2[u]][i1[u]] = make_double2(c1u * w00.x - q0.x, c1u * w00.y - q0.y);
                    W[i2[u]][j1[u]] = make_double2(r0.x + c1u * w01.x, r0.y + c1u * w01.y);
                    W[j2[u]][i1[u]] = make_double2(c1u * w10.x - q1.x, c1u * w10.y - q1.y);
                    W[j2[u]][j1[u]] = make_double2(r1.x + c1u * w11.x, r1.y + c1u * w11.y);
                }
            }
            prev = step;
            __syncthreads();
        }
        if (sweep + 1 < inner_max && block_scan<NB, NT>(G, zthr, tol2, red, &smask, mask) <= tol) break;
    }
    // the W threads still owe the last step
    if (!gthr && k > 0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int P1 = (tt + 256 * u) / NP;
            int i1, j1, i2, j2;
            pair_of(prev, P1, NB, i1, j1);
            pair_of(prev, (tt + 256 * u) % NP, NB, i2, j2);
            const double c1u = rc[(k - 1) & 1][P1];
            const double2 s1u = rs[(k - 1) & 1][P1];
            const double2 w00 = W[i2][i1], w01 = W[i2][j1];
            const double2 w10 = W[j2][i1], w11 = W[j2][j1];
            const double2 q0 = dmulc(s1u, w01), q1 = dmulc(s1u, w11);
            const double2 r0 = dmul(s1u, w00), r1 = dmul(s1u, w10);
            W[i2][i1] = make_double2(c1u * w00.x - q0.x, c1u * w00.y - q0.y);
            W[i2][j1] = make_double2(r0.x + c1u * w01.x, r0.y + c1u * w01.y);
            W[j2][i1] = make_double2(c1u * w10.x - q1.x, c1u * w10.y - q1.y);
            W[j2][j1] = make_double2(r1.x + c1u * w11.x, r1.y + c1u * w11.y);
        }
    }
    __syncthreads();
    C2<T>* wo = Wout + (size_t)pair * (NB * NB);
    for (int e = t; e < NB * NB; e += NT) {
        const int i = e % NB, j = e / NB;
        wo[i + NB * j] = from_d2<T>(W[i][j]);
    }
    if (t == 0) {
        skip[pair] = 0;
        atomicMax(&info->offmax_bits, (unsigned long long)__double_as_longlong(off0));
        atomicAdd(&info->rotations, 1);
        atomicAdd(&info->inner_steps, steps_done);
    }
}

// ------------------------------------------------------------- pair update
// 64-row slabs per work-group (measured at a 4096 x 4096 split: FP32 is
// fastest with one slab and the most work-groups, FP64 with four)
template <typename T> constexpr int update_slabs() { return sizeof(T) == 8 ? 4 : 1; }
// [x_p x_q] <- [x_p x_q] W for one 64-row slab of the pair's NB columns.  A
// column is rotated hundreds of times in one decomposition, so this product
// stays on the storage precision's own MFMA in every mode: rounding of W or X
// here accumulates in the state, while Gram rounding only perturbs angles.

template <typename T, int JB>
__global__ __launch_bounds__(256) void k_pair_update(C2<T>* __restrict__ X, int m, int N, int ld,
                                                     const int* __restrict__ colmap, int nb,
                                                     int round, const C2<T>* __restrict__ Wm,
                                                     const int* __restrict__ skip,
                                                     const int* __restrict__ halt) {
    constexpr int NB = 2 * JB, MB = NB / 32;
    const int pair = blockIdx.x;
    if (*halt || skip[pair]) return;
    __shared__ C2<T> Ws[NB][NB + 1];   // Ws[k][j] = W[k][j]
    __shared__ __align__(16) C2<T> Xt[NB][64 + 2];   // Xt[col][row], rows in 16-byte aligned pairs
    __shared__ int cols[NB];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    int p, q;
    pair_of(round, pair, nb, p, q);
    if (t < NB) {
        const int lj = (t < JB) ? p * JB + t : q * JB + (t - JB);
        cols[t] = (lj < N) ? colmap[lj] : -1;
    }
    const C2<T>* wsrc = Wm + (size_t)pair * (NB * NB);
    for (int e = t; e < NB * NB; e += 256) Ws[e % NB][e / NB] = wsrc[e];
    constexpr int kUpdateSlabs = update_slabs<T>();
    // W stays in LDS for kUpdateSlabs consecutive 64-row slabs; the next slab
    // is loaded into registers while the current one is multiplied
    // each lane moves 16 bytes: two FP32 rows or one FP64 row of a column
    constexpr int E = 16 / (int)sizeof(C2<T>), RU = 64 / E;   // rows per unit, units per column
    constexpr int LE = NB * RU / 256;
    using LV = typename GramLoad<T>::type;
    const bool even = (ld % E) == 0;
    auto gload = [&](int r0, int e) -> LV {
        const int row = (e % RU) * E, c = cols[e / RU];
        const C2<T>* src = X + (size_t)ld * (c >= 0 ? c : 0) + r0 + row;
        if constexpr (E == 2) {
            if (c >= 0 && even && r0 + row + 1 < m) return *reinterpret_cast<const float4*>(src);
            const float2 a = (c >= 0 && r0 + row < m) ? src[0] : make_float2(0.f, 0.f);
            const float2 b = (c >= 0 && r0 + row + 1 < m) ? src[1] : make_float2(0.f, 0.f);
            return make_float4(a.x, a.y, b.x, b.y);
        } else {
            return (c >= 0 && r0 + row < m) ? src[0] : make_double2(0.0, 0.0);
        }
    };
    LV pre[LE];
    __syncthreads();
    {
        const int r0 = blockIdx.y * kUpdateSlabs * 64;
#pragma unroll
        for (int r = 0; r < LE; ++r) pre[r] = gload(r0, t + 256 * r);
    }
    for (int slab = 0; slab < kUpdateSlabs; ++slab) {
        const int r0 = (blockIdx.y * kUpdateSlabs + slab) * 64;
        if (r0 >= m) break;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < LE; ++r) {
            const int e = t + 256 * r;
            *reinterpret_cast<LV*>(&Xt[e / RU][(e % RU) * E]) = pre[r];
        }
        __syncthreads();
        if (slab + 1 < kUpdateSlabs && r0 + 64 < m) {
            const int r1 = r0 + 64;
#pragma unroll
            for (int r = 0; r < LE; ++r) pre[r] = gload(r1, t + 256 * r);
        }
        // wave (wm, wn): rows wm*32 .. +32, columns wn*NB/2 .. +NB/2
        A4<T> accR[2][MB], accI[2][MB];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < MB; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) { accR[bi][bj][r] = T(0); accI[bi][bj][r] = T(0); }
#pragma unroll 4
        for (int kk = 0; kk < NB; kk += 4) {
            C2<T> a[2], b[MB];
#pragma unroll
            for (int s = 0; s < 2; ++s) a[s] = Xt[kk + (lane >> 4)][wm * 32 + s * 16 + (lane & 15)];
#pragma unroll
            for (int s = 0; s < MB; ++s) b[s] = Ws[kk + (lane >> 4)][wn * (NB / 2) + s * 16 + (lane & 15)];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < MB; ++bj) {
                    accR[bi][bj] = mfma16(a[bi].x, b[bj].x, accR[bi][bj]);
                    accR[bi][bj] = mfma16(-a[bi].y, b[bj].y, accR[bi][bj]);
                    accI[bi][bj] = mfma16(a[bi].x, b[bj].y, accI[bi][bj]);
                    accI[bi][bj] = mfma16(a[bi].y, b[bj].x, accI[bi][bj]);
                }
        }
        __syncthreads();
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < MB; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = wm * 32 + bi * 16 + acc_row<T>(lane, r);
                    const int col = wn * (NB / 2) + bj * 16 + (lane & 15);
                    Xt[col][row] = cmake<T>(accR[bi][bj][r], accI[bi][bj][r]);
                }
        __syncthreads();
        for (int e = t; e < NB * RU; e += 256) {
            const int row = (e % RU) * E, col = e / RU;
            const int c = cols[col];
            if (c < 0 || r0 + row >= m) continue;
            C2<T>* dst = X + (size_t)ld * c + r0 + row;
            if (E == 1 || (even && r0 + row + E - 1 < m)) {
                *reinterpret_cast<LV*>(dst) = *reinterpret_cast<const LV*>(&Xt[col][row]);
            } else {
                for (int u = 0; u < E; ++u)
                    if (r0 + row + u < m) dst[u] = Xt[col][row + u];
            }
        }
    }
}

// ------------------------------------------------------- truncation/entropy
// App. A truncation with a relative cutoff; entropy of Sec. III.C over the kept
// values.  Single work-group, FP64.
__global__ __launch_bounds__(256) void k_truncate(const double* __restrict__ sig2, int N,
                                                  int chi_max, double cutoff, double floor_rel2,
                                                  DevInfo* info, int with_rest) {
    __shared__ double red[256];
    __shared__ int cnt[256];
    __shared__ double s_total, s_kept;
    __shared__ int s_k;
    const int t = threadIdx.x;
    double part = 0.0;
    for (int e = t; e < N; e += 256) part += sig2[e];
    red[t] = part;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    // values left out of sig2 (all below the last of it) count as discarded
    const double rest = with_rest ? info->rest_weight : 0.0;
    if (t == 0) s_total = red[0] + rest;
    __syncthreads();
    const double total = s_total;
    // values the sweep treated as zero are never kept
    const double thr = fmax(cutoff * cutoff, floor_rel2) * total;
    int c = 0;
    for (int e = t; e < N; e += 256) c += (sig2[e] > thr) ? 1 : 0;
    cnt[t] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) cnt[t] += cnt[t + o];
        __syncthreads();
    }
    if (t == 0) {
        int k = cnt[0];
        if (k > chi_max) k = chi_max;
        if (k > N) k = N;
        if (k < 1) k = 1;
        s_k = k;
    }
    __syncthreads();
    const int k = s_k;
    double kp = 0.0, dp = 0.0;
    for (int e = t; e < N; e += 256) {
        if (e < k) kp += sig2[e]; else dp += sig2[e];
    }
    red[t] = kp;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    if (t == 0) s_kept = red[0];
    __syncthreads();
    const double kept = s_kept;
    __syncthreads();
    red[t] = dp;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    const double disc = red[0] + rest;
    __syncthreads();
    double ent = 0.0;
    if (kept > 0.0) {
        for (int e = t; e < k; e += 256) {
            const double w = sig2[e] / kept;
            if (w > 0.0) ent -= w * log2(w);
        }
    }
    red[t] = ent;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    if (t == 0) {
        info->kept = k;
        info->total = total;
        info->discarded = disc;
        info->entropy = red[0];
        info->numeric_error = (isfinite(total) && isfinite(red[0])) ? 0 : 1;
    }
}

// ------------------------------------------------------------------ gathers
template <typename T>
__global__ void k_gather_cols(const C2<T>* __restrict__ X, int m, int ld, const int* __restrict__ colmap,
                              const double* __restrict__ sig2, int k, C2<T>* __restrict__ dst,
                              int ldd, int normalize) {
    const int b = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= k || i >= m) return;
    const double s2 = sig2[b];
    C2<T> v;
    if (!normalize) {
        v = X[(size_t)i + (size_t)ld * colmap[b]];
    } else if (s2 > 0.0) {
        const double inv = 1.0 / sqrt(s2);
        const double2 x = to_d2(X[(size_t)i + (size_t)ld * colmap[b]]);
        v = cmake<T>(T(x.x * inv), T(x.y * inv));
    } else {
        v = cmake<T>(T(i == b ? 1 : 0), T(0));
    }
    dst[(size_t)i + (size_t)ldd * b] = v;
}

template <typename T>
__global__ void k_gather_rows_conj(const C2<T>* __restrict__ X, int m, int ld,
                                   const int* __restrict__ colmap,
                                   const double* __restrict__ sig2, int k,
                                   C2<T>* __restrict__ dst) {
    __shared__ C2<T> tile[32][33];
    const int i0 = blockIdx.x * 32, b0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: ty 0..7
    for (int r = ty; r < 32; r += 8) {
        const int b = b0 + r, i = i0 + tx;
        C2<T> v = czero<T>();
        if (b < k && i < m) {
            const double s2 = sig2[b];
            if (s2 > 0.0) {
                const double inv = 1.0 / sqrt(s2);
                const double2 x = to_d2(X[(size_t)i + (size_t)ld * colmap[b]]);
                v = cmake<T>(T(x.x * inv), T(-x.y * inv));
            } else {
                v = cmake<T>(T(i == b ? 1 : 0), T(0));
            }
        }
        tile[r][tx] = v;   // tile[b][i]
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + r, b = b0 + tx;
        if (b < k && i < m) dst[(size_t)b + (size_t)k * i] = tile[tx][r];
    }
}

template <typename T>
__global__ void k_conj_transpose(const C2<T>* __restrict__ A, int rows, int cols, int lda,
                                 C2<T>* __restrict__ Y, int ldy) {
    __shared__ C2<T> tile[32][33];
    const int r0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int i = r0 + tx, j = c0 + r;
        if (i < rows && j < cols) tile[r][tx] = cconj<T>(A[(size_t)i + (size_t)lda * j]);
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int j = c0 + tx, i = r0 + r;
        if (i < rows && j < cols) Y[(size_t)j + (size_t)ldy * i] = tile[tx][r];
    }
}

// dst[i + ldd * j] = src[i + lds * j] for a rows x cols block
template <typename T>
__global__ void k_copy_cols(const C2<T>* __restrict__ src, int rows, int lds, C2<T>* __restrict__ dst,
                            int ldd) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i < rows) dst[(size_t)i + (size_t)ldd * j] = src[(size_t)i + (size_t)lds * j];
}

template <typename T>
__global__ void k_copy(const C2<T>* __restrict__ s, C2<T>* __restrict__ d, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}

// Power-of-two scaling of X in the FP32-storage modes.  FP32 products of
// entries far below 1 leave the normal range (a state of total weight 1e-27 has
// entries near 1e-17, whose products are denormal or zero), which corrupts the
// Gram of the small columns and stalls the sweeps.  Before the first sweep X
// is scaled by 2^k, k chosen from ||X||_F so that the scaled norm lies in
// [1/2, 1); after the last one the factor is removed from X, the sorted squared
// norms and ||X||_F^2.  Scaling by a power of two is exact.
__global__ void k_scale_exp(DevInfo* info, double* fro2, int undo) {
    if (threadIdx.x != 0) return;
    if (!undo) {
        int e = 0;
        const double f = *fro2;
        if (f > 0.0 && isfinite(f)) (void)frexp(sqrt(f), &e);
        info->scale_exp = -e;
        *fro2 = ldexp(f, -2 * e);
    } else {
        *fro2 = ldexp(*fro2, -2 * info->scale_exp);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_scale_apply(C2<T>* __restrict__ X, size_t n,
                                                     const DevInfo* __restrict__ info,
                                                     double* __restrict__ sig2, int N, int undo) {
    const int k = undo ? -info->scale_exp : info->scale_exp;
    if (k == 0) return;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        C2<T> v = X[i];
        v.x = ldexp(v.x, k);
        v.y = ldexp(v.y, k);
        X[i] = v;
    }
    if (undo && sig2)
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)N; i += stride)
            sig2[i] = ldexp(sig2[i], 2 * k);
}

// Start of a sweep: clear the sweep's measures (no memset node, so that a
// captured sweep replays correctly).  End of a sweep: the convergence test on
// the device, so that sweeps can be queued ahead of the host's read.
__global__ void k_sweep_begin(DevInfo* info) {
    if (threadIdx.x != 0 || info->done) return;
    info->offmax_bits = 0ull;
    info->rotations = 0;
    info->inner_steps = 0;
}

__global__ void k_sweep_end(DevInfo* info, double stop_off, int max_sweeps) {
    if (threadIdx.x != 0 || info->done) return;
    const double off = __longlong_as_double((long long)info->offmax_bits);
    info->sweeps += 1;
    info->rot_total += info->rotations;
    if (info->rotations == 0 || off <= stop_off) info->done = 1;
    else if (info->sweeps >= max_sweeps) info->done = 2;
}

__global__ void k_jacobi_reset(DevInfo* info) {
    if (threadIdx.x != 0) return;
    info->done = 0;
    info->sweeps = 0;
    info->rot_total = 0;
}

// ------------------------------------------------------------------- host side
// Captured sweeps, one per shape, owned by the handle.
struct SweepGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};
using GraphKey = std::tuple<int, int, int, int, int, int, long, long>;
using GraphCache = std::map<GraphKey, SweepGraph>;

void* jacobi_graph_cache_new() { return new GraphCache(); }
void jacobi_graph_cache_free(void* cache) {
    GraphCache* c = (GraphCache*)cache;
    if (!c) return;
    for (auto& kv : *c) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    delete c;
}

template <typename T, int JB, bool BF>
static int jacobi_run(C2<T>* X, int m, int N, int ld, double tol, double stop_off, double zrel2,
                      int max_sweeps, int inner_max, JacobiWork& w, hipStream_t st) {
    constexpr int NB = 2 * JB;
    int nb = (N + JB - 1) / JB;
    if (nb < 2) nb = 2;
    if (nb & 1) ++nb;
    const int P = nb / 2;
    if ((size_t)P * NB * NB > (size_t)w.max_pairs * 4096 || P > 4 * w.max_pairs) return -3;
    int splits = (512 + P - 1) / P;
    if (splits > w.splits) splits = w.splits;
    constexpr int RB = 4096 / NB;
    int chunk = (m + splits - 1) / splits;
    chunk = (chunk + RB - 1) / RB * RB;
    splits = (m + chunk - 1) / chunk;
    if (splits < 1) splits = 1;
    double* fro2 = &w.info->total;   // scratch slot reused for ||X||_F^2
    const int* halt = &w.info->done;
    const dim3 gnorm((N + 3) / 4);
    Profiler& pf = *w.prof;
    const double csz = 2.0 * sizeof(T);
    const double pair_flops = 8.0 * m * NB * NB;      // one NB x NB complex product over m rows
    // the Gram kernels form only the TB(TB+1)/2 upper 16x16 tiles of the Hermitian
    // NB x NB product (TB = NB/16): credit those tiles, not the full product
    constexpr int kTB = NB / 16, kNU = kTB * (kTB + 1) / 2;
    const double gram_flops = 8.0 * m * 256.0 * kNU;
    const double pair_bytes = (double)m * NB * csz;
    // FP32 storage: X is held scaled by a power of two during the sweeps
    constexpr bool scaled = sizeof(T) == 4;
    const dim3 gscale((unsigned)std::min<size_t>(2048, ((size_t)ld * N + 255) / 256));
    auto unscale = [&](bool with_values) {
        if (!scaled) return;
        hipLaunchKernelGGL((k_scale_apply<T>), gscale, dim3(256), 0, st, X, (size_t)ld * N,
                           (const DevInfo*)w.info, with_values ? w.sig2 : (double*)nullptr, N, 1);
        hipLaunchKernelGGL(k_scale_exp, dim3(1), dim3(64), 0, st, w.info, fro2, 1);
    };
    // One sweep: norm sort, then nb-1 rounds of (pair Gram, pair eigen-solver,
    // pair update), then the convergence test on the device.  Every launch
    // returns at once when an earlier sweep already converged, so sweeps may be
    // queued ahead of the host's read.  Per-launch events (profiling) are
    // recorded only when the sweep is not being captured.
    auto enqueue_sweep = [&](bool events, int sweep_limit) {
        if (events) pf.begin(st);
        hipLaunchKernelGGL((k_colnorm2<T>), gnorm, dim3(256), 0, st, X, m, N, ld, w.nrm2, halt);
        hipLaunchKernelGGL(k_sort_desc, dim3(1), dim3(1024), 0, st, w.nrm2, N, w.colmap, w.sig2, fro2, halt);
        if (events) pf.end(st, K_NORMSORT, 8.0 * m * N, (double)m * N * csz);
        hipLaunchKernelGGL(k_sweep_begin, dim3(1), dim3(64), 0, st, w.info);
        for (int r = 0; r < nb - 1; ++r) {
            hipEvent_t a = nullptr, b = nullptr;
            // timed launches carry start/stop events; plain ones can be captured
#define MPO_LAUNCH(K, G, B, ...)                                                      \
    do {                                                                              \
        if (events) hipExtLaunchKernelGGL(K, G, B, 0, st, a, b, 0, __VA_ARGS__);      \
        else hipLaunchKernelGGL(K, G, B, 0, st, __VA_ARGS__);                         \
    } while (0)
            if (events) pf.stamps(a, b);
            if constexpr (BF)
                MPO_LAUNCH((k_pair_gram_bf3<JB>), dim3(P, splits), dim3(256), X, m, N, ld,
                           (const int*)w.colmap, nb, r, splits, chunk, (double2*)w.gram_partials, halt);
            else if constexpr (sizeof(T) == 4)
                MPO_LAUNCH((k_pair_gram_regs<T, JB>), dim3(P, splits), dim3(256), X, m, N, ld,
                           (const int*)w.colmap, nb, r, splits, chunk, (double2*)w.gram_partials, halt);
            else
                MPO_LAUNCH((k_pair_gram_lds<T, JB>), dim3(P, splits), dim3(256), X, m, N, ld,
                           (const int*)w.colmap, nb, r, splits, chunk, (double2*)w.gram_partials, halt);
            if (events) pf.record(K_GRAM, a, b, P * gram_flops, P * pair_bytes + (double)P * splits * NB * NB * 16.0);
            if (events) pf.stamps(a, b);
            MPO_LAUNCH((k_pair_eig<T, JB>), dim3(P), dim3(kEigThreads), (const double2*)w.gram_partials,
                       splits, tol, zrel2, (const double*)fro2, inner_max, (C2<T>*)w.w, w.skip, w.info);
            if (events) pf.record(K_EIG, a, b, 0.0, (double)P * splits * NB * NB * 16.0);
            constexpr int US = update_slabs<T>();
            if (events) pf.stamps(a, b);
            MPO_LAUNCH((k_pair_update<T, JB>), dim3(P, (m + 64 * US - 1) / (64 * US)), dim3(256), X, m, N,
                       ld, (const int*)w.colmap, nb, r, (const C2<T>*)w.w, (const int*)w.skip, halt);
            if (events) pf.record(K_UPDATE, a, b, 0.0, 0.0);
#undef MPO_LAUNCH
        }
        hipLaunchKernelGGL(k_sweep_end, dim3(1), dim3(64), 0, st, w.info, stop_off, sweep_limit);
    };
    auto read_info = [&]() -> bool {
        if (hipMemcpyAsync(w.info_host, w.info, sizeof(DevInfo), hipMemcpyDeviceToHost, st) != hipSuccess)
            return false;
        return hipStreamSynchronize(st) == hipSuccess;
    };
    // norms, order and (FP32 storage) the power-of-two scale before the first sweep
    hipLaunchKernelGGL(k_jacobi_reset, dim3(1), dim3(64), 0, st, w.info);
    pf.begin(st);
    hipLaunchKernelGGL((k_colnorm2<T>), gnorm, dim3(256), 0, st, X, m, N, ld, w.nrm2, (const int*)nullptr);
    hipLaunchKernelGGL(k_sort_desc, dim3(1), dim3(1024), 0, st, w.nrm2, N, w.colmap, w.sig2, fro2,
                       (const int*)nullptr);
    if (scaled) {
        hipLaunchKernelGGL(k_scale_exp, dim3(1), dim3(64), 0, st, w.info, fro2, 0);
        hipLaunchKernelGGL((k_scale_apply<T>), gscale, dim3(256), 0, st, X, (size_t)ld * N,
                           (const DevInfo*)w.info, (double*)nullptr, N, 0);
    }
    pf.end(st, K_NORMSORT, 8.0 * m * N, (double)m * N * csz);
    int done = 0, sweeps = 0;
    if (w.graphs && st != nullptr && !pf.on) {
        // captured sweeps, replayed in batches between host reads; the batch
        // size follows the sweeps the last decomposition of this shape needed
        GraphCache& cache = *(GraphCache*)w.graph_cache;
        // the captured launches carry the shape, tol and stop_off (the sweep
        // limit is checked here, between batches)
        const GraphKey key = std::make_tuple(m, N, ld, JB, (int)BF, (int)sizeof(T),
                                             (long)std::llround(std::log10(stop_off) * 1000.0),
                                             (long)std::llround(std::log10(tol) * 1000.0));
        SweepGraph& sg = cache[key];
        if (!sg.exec) {
            if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return -2;
            enqueue_sweep(false, 1 << 30);
            if (hipStreamEndCapture(st, &sg.graph) != hipSuccess) return -2;
            if (hipGraphInstantiate(&sg.exec, sg.graph, nullptr, nullptr, 0) != hipSuccess) return -2;
        }
        static thread_local std::map<GraphKey, int> last_sweeps;
        int batch = std::max(2, last_sweeps.count(key) ? last_sweeps[key] : 4);
        while (!done) {
            batch = std::min(batch, max_sweeps - sweeps);
            if (batch <= 0) { done = 2; break; }
            for (int q = 0; q < batch; ++q)
                if (hipGraphLaunch(sg.exec, st) != hipSuccess) return -2;
            if (!read_info()) return -2;
            done = w.info_host->done;
            sweeps = w.info_host->sweeps;
            batch = 2;
        }
        last_sweeps[key] = sweeps;
        w.n_rotations += w.info_host->rot_total;
    } else {
        for (;;) {
            enqueue_sweep(pf.on, max_sweeps);
            if (!read_info()) return -2;
            done = w.info_host->done;
            sweeps = w.info_host->sweeps;
            const unsigned long long bits = w.info_host->offmax_bits;
            double off;
            std::memcpy(&off, &bits, sizeof(off));
            const int rot = w.info_host->rotations;
            w.n_rotations += rot;
            if (w.trace)
                std::fprintf(stderr, "jacobi %dx%d sweep %d: max rel off-diagonal %.3e, %d of %d pairs x %d rounds rotated\n",
                             m, N, sweeps - 1, off, rot, P, nb - 1);
            pf.add_work(K_UPDATE, rot * pair_flops, rot * 2.0 * pair_bytes);
            // each inner step applies a two-sided 2x2 transform to all NB^2 entries of G
            // (22 real flops per entry) and a column rotation to W (11 per entry)
            pf.add_work(K_EIG, 33.0 * NB * NB * (double)w.info_host->inner_steps, 0.0);
            if (done) break;
        }
    }
    w.n_rounds += (long long)sweeps * (nb - 1);
    w.n_sweeps += sweeps;
    if (done != 1) {
        unscale(false);
        return -1;
    }
    pf.begin(st);
    hipLaunchKernelGGL((k_colnorm2<T>), gnorm, dim3(256), 0, st, X, m, N, ld, w.nrm2, (const int*)nullptr);
    hipLaunchKernelGGL(k_sort_desc, dim3(1), dim3(1024), 0, st, w.nrm2, N, w.colmap, w.sig2, fro2,
                       (const int*)nullptr);
    unscale(true);
    pf.end(st, K_NORMSORT, 8.0 * m * N, (double)m * N * csz);
    return sweeps;
}

// Sweeps stop when no pair rotated or when the largest relative off-diagonal
// met at the start of the pairs is at most stop_off (= tol, except for the
// first phase of split-BF16x3 mode).
template <typename T>
int jacobi_orthogonalize(C2<T>* X, int m, int N, int ld, double tol, int max_sweeps, JacobiWork& w,
                         hipStream_t st, int keep_max) {
    w.n_splits += 1;
    w.n_cols = N;
    w.rest_on = false;
    // Start from the eigenvectors of X^H X: the columns are then orthogonal to
    // about the FP64 eigen-solver's accuracy and the sweeps only polish.
    bool started = false;
    if (w.heev && w.precond_min > 0 && N >= w.precond_min && N <= w.heev->cap_n && m <= w.heev->cap_m) {
        // A caller keeping at most keep_max columns: only the eigenvectors of the
        // largest keep_max + 64 eigenvalues (rounded up to 64) are applied.  Their
        // span is the leading singular subspace up to rotations into the left-out
        // directions of size u ||G|| / (lambda_keep_max - lambda_keep), which the
        // 64-column margin keeps far from the kept values; those rotations change
        // the kept singular values only at second order.  Within the span the
        // certificate (FP32 storage) or the sweeps (FP64) finish the columns.
        int keep = N;
        if (keep_max > 0) {
            const int k2 = (keep_max + 64 + 63) / 64 * 64;
            if (2 * k2 <= N) keep = k2;
        }
        const int ncols = heev_precondition<T>(X, m, N, ld, keep, &w.info->rest_weight, *w.heev, *w.prof, st);
        if (ncols < N) {
            N = ncols;
            w.n_cols = N;
            w.rest_on = true;
        }
        w.n_precond += 1;
        started = true;
        // FP32 storage: the start is orthogonal to well below the sweeps' FP32
        // tolerance, so one FP64 Gram product certifies it in place of a sweep
        // that would find nothing to rotate; only norms and order remain.  (In
        // FP64 storage the start is left to the sweeps: its small columns are
        // only as orthogonal as the Gram's absolute accuracy allows.)
        if (sizeof(T) == 4 &&
            heev_check<T>(X, m, N, ld, std::fmin(tol, kTolFp32), jacobi_zero_rel2<T>(), w.info, w.info_host,
                          *w.heev, *w.prof, st)) {
            hipLaunchKernelGGL(k_jacobi_reset, dim3(1), dim3(64), 0, st, w.info);
            double* fro2 = &w.info->total;
            w.prof->begin(st);
            hipLaunchKernelGGL((k_colnorm2<T>), dim3((N + 3) / 4), dim3(256), 0, st, X, m, N, ld, w.nrm2,
                               (const int*)nullptr);
            hipLaunchKernelGGL(k_sort_desc, dim3(1), dim3(1024), 0, st, w.nrm2, N, w.colmap, w.sig2, fro2,
                               (const int*)nullptr);
            w.prof->end(st, K_NORMSORT, 8.0 * m * N, (double)m * N * 2.0 * sizeof(T));
            w.n_checks += 1;
            return 0;
        }
    }
    if constexpr (sizeof(T) == 4) {
        if (w.bf3 && !started) {
            // BF16x3 Gram until a sweep starts within kBf3Handoff of orthogonal
            // (convergence is quadratic there, so it ends near 1e-5), then the
            // FP32-MFMA Gram down to kTolFp32; both with the BF16x3 zero floor
            const double hand = std::fmax(tol, kBf3Handoff);
            const int s1 = w.block == 16
                ? jacobi_run<T, 16, true>(X, m, N, ld, tol, hand, kZeroRel2Bf3, max_sweeps, w.inner, w, st)
                : jacobi_run<T, 32, true>(X, m, N, ld, tol, hand, kZeroRel2Bf3, max_sweeps, w.inner, w, st);
            if (s1 < 0 || tol <= kTolFp32) return s1;
            const int s2 = w.block == 16
                ? jacobi_run<T, 16, false>(X, m, N, ld, kTolFp32, kTolFp32, kZeroRel2Bf3, max_sweeps - s1,
                                           w.inner, w, st)
                : jacobi_run<T, 32, false>(X, m, N, ld, kTolFp32, kTolFp32, kZeroRel2Bf3, max_sweeps - s1,
                                           w.inner, w, st);
            return s2 < 0 ? s2 : s1 + s2;
        }
    }
    const double zrel2 = jacobi_zero_rel2<T>();
    // split-BF16x3 from the eigen-solver's start: only the FP32-Gram polish remains
    if (sizeof(T) == 4 && w.bf3) tol = std::fmin(tol, kTolFp32);
    if (w.block == 16) return jacobi_run<T, 16, false>(X, m, N, ld, tol, tol, zrel2, max_sweeps, w.inner, w, st);
    return jacobi_run<T, 32, false>(X, m, N, ld, tol, tol, zrel2, max_sweeps, w.inner, w, st);
}

void launch_truncate(const double* sig2, int N, int chi_max, double cutoff, double floor_rel2,
                     DevInfo* info, hipStream_t st, bool with_rest) {
    hipLaunchKernelGGL(k_truncate, dim3(1), dim3(256), 0, st, sig2, N, chi_max, cutoff, floor_rel2,
                       info, (int)with_rest);
}

template <typename T>
void launch_gather_cols(const C2<T>* X, int m, int ldx, const int* colmap, const double* sig2, int k,
                        C2<T>* dst, int ldd, hipStream_t st, bool normalize) {
    hipLaunchKernelGGL((k_gather_cols<T>), dim3((m + 255) / 256, k), dim3(256), 0, st, X, m, ldx, colmap,
                       sig2, k, dst, ldd, normalize ? 1 : 0);
}
template <typename T>
void launch_gather_rows_conj(const C2<T>* X, int m, int ldx, const int* colmap, const double* sig2,
                             int k, C2<T>* dst, hipStream_t st) {
    hipLaunchKernelGGL((k_gather_rows_conj<T>), dim3((m + 31) / 32, (k + 31) / 32), dim3(256), 0, st,
                       X, m, ldx, colmap, sig2, k, dst);
}
template <typename T>
void launch_conj_transpose(const C2<T>* A, int rows, int cols, int lda, C2<T>* Y, int ldy,
                           hipStream_t st) {
    hipLaunchKernelGGL((k_conj_transpose<T>), dim3((rows + 31) / 32, (cols + 31) / 32), dim3(256), 0,
                       st, A, rows, cols, lda, Y, ldy);
}
template <typename T>
void launch_copy_cols(const C2<T>* src, int rows, int cols, int lds, C2<T>* dst, int ldd, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return;
    hipLaunchKernelGGL((k_copy_cols<T>), dim3((rows + 255) / 256, cols), dim3(256), 0, st, src, rows, lds,
                       dst, ldd);
}
template <typename T>
void launch_copy(const C2<T>* src, C2<T>* dst, size_t count, hipStream_t st) {
    if (!count) return;
    hipLaunchKernelGGL((k_copy<T>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, src, dst, count);
}

#define INST(T)                                                                                  \
    template int jacobi_orthogonalize<T>(C2<T>*, int, int, int, double, int, JacobiWork&, hipStream_t, int); \
    template void launch_gather_cols<T>(const C2<T>*, int, int, const int*, const double*, int,     \
                                        C2<T>*, int, hipStream_t, bool);                           \
    template void launch_gather_rows_conj<T>(const C2<T>*, int, int, const int*, const double*, int, \
                                             C2<T>*, hipStream_t);                                 \
    template void launch_conj_transpose<T>(const C2<T>*, int, int, int, C2<T>*, int, hipStream_t); \
    template void launch_copy_cols<T>(const C2<T>*, int, int, int, C2<T>*, int, hipStream_t);      \
    template void launch_copy<T>(const C2<T>*, C2<T>*, size_t, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace mpo

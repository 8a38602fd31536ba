// Transfer contraction of the vectorised MPO with one 4-vector per site
// (Sec. III.D: total probability and output probabilities as a chain of
// vector-matrix products).  Environments are FP64 complex in every precision.
#include "common.h"

namespace mpo {

// env_out[b] = sum_{I,a} env_in[a] v[I] A[a + chiL*(I + 4b)]: one work-group
// per output b, reducing over the contiguous 4*chiL entries of column b.
template <typename T>
__global__ __launch_bounds__(256) void k_transfer_left(const C2<T>* __restrict__ A, int chiL,
                                                       int chiR, const double2* __restrict__ env,
                                                       const double2* __restrict__ v,
                                                       double2* __restrict__ out) {
    __shared__ double2 red[256];
    const int b = blockIdx.x, t = threadIdx.x;
    const int len = 4 * chiL;
    const C2<T>* col = A + (size_t)len * b;
    double sr = 0.0, si = 0.0;
    for (int e = t; e < len; e += 256) {
        const int a = e % chiL, I = e / chiL;
        const double2 x = to_d2(col[e]);
        const double2 ev = env[a], vv = v[I];
        const double2 w = make_double2(ev.x * vv.x - ev.y * vv.y, ev.x * vv.y + ev.y * vv.x);
        sr += w.x * x.x - w.y * x.y;
        si += w.x * x.y + w.y * x.x;
    }
    red[t] = make_double2(sr, si);
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) { red[t].x += red[t + o].x; red[t].y += red[t + o].y; }
        __syncthreads();
    }
    if (t == 0) out[b] = red[0];
}

// Partial right transfer: scratch[chunk*chiL + a] = sum over this chunk's
// (I, b) of A[a + chiL*(I + 4b)] v[I] env_in[b]; thread per a (coalesced).
template <typename T>
__global__ __launch_bounds__(256) void k_transfer_right_part(const C2<T>* __restrict__ A, int chiL,
                                                             int chiR, const double2* __restrict__ env,
                                                             const double2* __restrict__ v,
                                                             int per_chunk,
                                                             double2* __restrict__ scratch) {
    const int a = blockIdx.x * 256 + threadIdx.x;
    const int chunk = blockIdx.y;
    if (a >= chiL) return;
    const int j0 = chunk * per_chunk, j1 = min(4 * chiR, j0 + per_chunk);
    double sr = 0.0, si = 0.0;
    for (int j = j0; j < j1; ++j) {      // j = I + 4b
        const int I = j & 3, b = j >> 2;
        const double2 x = to_d2(A[(size_t)a + (size_t)chiL * j]);
        const double2 ev = env[b], vv = v[I];
        const double2 w = make_double2(ev.x * vv.x - ev.y * vv.y, ev.x * vv.y + ev.y * vv.x);
        sr += w.x * x.x - w.y * x.y;
        si += w.x * x.y + w.y * x.x;
    }
    scratch[(size_t)chunk * chiL + a] = make_double2(sr, si);
}

__global__ void k_sum_chunks(const double2* __restrict__ scratch, int chiL, int chunks,
                             double2* __restrict__ out) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= chiL) return;
    double sr = 0.0, si = 0.0;
    for (int c = 0; c < chunks; ++c) {
        sr += scratch[(size_t)c * chiL + a].x;
        si += scratch[(size_t)c * chiL + a].y;
    }
    out[a] = make_double2(sr, si);
}

__global__ __launch_bounds__(256) void k_dot(const double2* __restrict__ x,
                                             const double2* __restrict__ y, int len,
                                             double2* __restrict__ out) {
    __shared__ double2 red[256];
    const int t = threadIdx.x;
    double sr = 0.0, si = 0.0;
    for (int e = t; e < len; e += 256) {
        const double2 a = x[e], b = y[e];
        sr += a.x * b.x - a.y * b.y;
        si += a.x * b.y + a.y * b.x;
    }
    red[t] = make_double2(sr, si);
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) { red[t].x += red[t + o].x; red[t].y += red[t + o].y; }
        __syncthreads();
    }
    if (t == 0) *out = red[0];
}

// Local gradient of a bilinear form: out[4I+J][4K+L] =
//   sum_{a,c} conj(X[(I,a),(J,c)]) Y[(K,a),(L,c)]
// for two (4 chiA) x (4 chiC) column-major two-site blocks (row a + chiA*I,
// column J + 4c).  One work-group per output entry, FP64 accumulation.
template <typename T>
__global__ __launch_bounds__(256) void k_local_grad(const C2<T>* __restrict__ X,
                                                    const C2<T>* __restrict__ Y, int chiA,
                                                    int chiC, double2* __restrict__ out) {
    __shared__ double2 red[256];
    const int o = blockIdx.x, t = threadIdx.x;
    const int I = o >> 6, J = (o >> 4) & 3, K = (o >> 2) & 3, L = o & 3;
    const size_t ld = 4 * (size_t)chiA;
    double sr = 0.0, si = 0.0;
    const int total = chiA * chiC;
    for (int e = t; e < total; e += 256) {
        const int a = e % chiA, c = e / chiA;
        const double2 x = to_d2(X[(size_t)(a + chiA * I) + ld * (J + 4 * c)]);
        const double2 y = to_d2(Y[(size_t)(a + chiA * K) + ld * (L + 4 * c)]);
        sr += x.x * y.x + x.y * y.y;
        si += x.x * y.y - x.y * y.x;
    }
    red[t] = make_double2(sr, si);
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) { red[t].x += red[t + s].x; red[t].y += red[t + s].y; }
        __syncthreads();
    }
    if (t == 0) out[(4 * I + J) * 16 + (4 * K + L)] = red[0];
}

// One site of sequential conditional sampling (Sec. III.D, sampling via
// marginals), one work-group per sample s.  Ybar[(I + 4c) + 4 chiR s] holds
// conj of the prefix environment times the site tensor (computed as A^H Lbar by
// the GEMM), Rk[c] the sites to the right summed out.  The marginals of the
// two candidate dits are q_b = sum_c (sum_I v_b[I] Y[I + 4c]) Rk[c]; negative
// ones are taken as 0 (flagged), the dit is 0 when u < p0 / (p0 + p1), and the
// new environment conj(T_x) / (p0 + p1) keeps its scale near 1 (log of the
// scale accumulated in logN).  v holds v_0[0..3] then v_1[0..3].
template <typename T>
__global__ __launch_bounds__(256) void k_sample_site(const C2<T>* __restrict__ Ybar, int chiR,
                                                     const double2* __restrict__ Rk,
                                                     const double2* __restrict__ v,
                                                     const double* __restrict__ u, int n, int site,
                                                     C2<T>* __restrict__ Lnew,
                                                     unsigned char* __restrict__ bits,
                                                     double* __restrict__ logN,
                                                     int* __restrict__ clamped) {
    __shared__ double red[4][256];
    __shared__ double s_scale;
    __shared__ int s_x;
    const int t = threadIdx.x, smp = blockIdx.x;
    const C2<T>* y = Ybar + (size_t)4 * chiR * smp;
    double2 vv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) vv[k] = v[k];
    double q0r = 0.0, q0i = 0.0, q1r = 0.0, q1i = 0.0;
    for (int c = t; c < chiR; c += 256) {
        double2 t0 = make_double2(0.0, 0.0), t1 = make_double2(0.0, 0.0);
#pragma unroll
        for (int I = 0; I < 4; ++I) {
            const double2 yb = to_d2(y[I + 4 * c]);
            const double2 yi = make_double2(yb.x, -yb.y);
            t0.x += vv[I].x * yi.x - vv[I].y * yi.y;
            t0.y += vv[I].x * yi.y + vv[I].y * yi.x;
            t1.x += vv[4 + I].x * yi.x - vv[4 + I].y * yi.y;
            t1.y += vv[4 + I].x * yi.y + vv[4 + I].y * yi.x;
        }
        const double2 r = Rk[c];
        q0r += t0.x * r.x - t0.y * r.y;
        q0i += t0.x * r.y + t0.y * r.x;
        q1r += t1.x * r.x - t1.y * r.y;
        q1i += t1.x * r.y + t1.y * r.x;
    }
    red[0][t] = q0r;
    red[1][t] = q1r;
    red[2][t] = q0i;
    red[3][t] = q1i;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) {
#pragma unroll
            for (int k = 0; k < 4; ++k) red[k][t] += red[k][t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        const double q0 = red[0][0], q1 = red[1][0];
        if (q0 < 0.0 || q1 < 0.0) clamped[smp] = 1;
        const double p0 = fmax(q0, 0.0), p1 = fmax(q1, 0.0), tot = p0 + p1;
        const int x = (tot == 0.0 || u[(size_t)smp * n + site] < p0 / tot) ? 0 : 1;
        bits[(size_t)smp * n + site] = (unsigned char)x;
        const double scale = tot > 0.0 ? tot : 1.0;
        logN[smp] += log(scale);
        s_scale = scale;
        s_x = x;
    }
    __syncthreads();
    const double inv = 1.0 / s_scale;
    const int off = 4 * s_x;
    for (int c = t; c < chiR; c += 256) {
        double2 tx = make_double2(0.0, 0.0);
#pragma unroll
        for (int I = 0; I < 4; ++I) {
            const double2 yb = to_d2(y[I + 4 * c]);
            const double2 yi = make_double2(yb.x, -yb.y);
            tx.x += vv[off + I].x * yi.x - vv[off + I].y * yi.y;
            tx.y += vv[off + I].x * yi.y + vv[off + I].y * yi.x;
        }
        Lnew[(size_t)c + (size_t)chiR * smp] = cmake<T>(T(tx.x * inv), T(-tx.y * inv));
    }
}

template <typename T>
__global__ void k_sample_init(C2<T>* __restrict__ L, double* __restrict__ logN,
                              int* __restrict__ clamped, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    L[i] = cmake<T>(T(1), T(0));
    logN[i] = 0.0;
    clamped[i] = 0;
}

template <typename T>
void launch_sample_init(C2<T>* L, double* logN, int* clamped, int count, hipStream_t st) {
    hipLaunchKernelGGL((k_sample_init<T>), dim3((count + 255) / 256), dim3(256), 0, st, L, logN,
                       clamped, count);
}
template <typename T>
void launch_sample_site(const C2<T>* Ybar, int chiR, int count, const double2* Rk, const double2* v,
                        const double* u, int n, int site, C2<T>* Lnew, unsigned char* bits,
                        double* logN, int* clamped, hipStream_t st) {
    hipLaunchKernelGGL((k_sample_site<T>), dim3(count), dim3(256), 0, st, Ybar, chiR, Rk, v, u, n,
                       site, Lnew, bits, logN, clamped);
}
template void launch_sample_init<double>(double2*, double*, int*, int, hipStream_t);
template void launch_sample_init<float>(float2*, double*, int*, int, hipStream_t);
template void launch_sample_site<double>(const double2*, int, int, const double2*, const double2*,
                                         const double*, int, int, double2*, unsigned char*, double*,
                                         int*, hipStream_t);
template void launch_sample_site<float>(const float2*, int, int, const double2*, const double2*,
                                        const double*, int, int, float2*, unsigned char*, double*,
                                        int*, hipStream_t);

// A[a, I, b] = [b == a + chiA*I] for a (chiA, 4, 4 chiA) site tensor.
template <typename T>
__global__ void k_identity_site(C2<T>* __restrict__ A, int chiA) {
    const size_t total = 16 * (size_t)chiA * chiA;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const size_t a_I = e % (4 * (size_t)chiA), b = e / (4 * (size_t)chiA);   // a + chiA*I, b
    A[e] = cmake<T>(T(a_I == b ? 1 : 0), T(0));
}

template <typename T>
void launch_identity_site(C2<T>* A, int chiA, hipStream_t st) {
    const size_t total = 16 * (size_t)chiA * chiA;
    hipLaunchKernelGGL((k_identity_site<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, A, chiA);
}
template void launch_identity_site<double>(double2*, int, hipStream_t);
template void launch_identity_site<float>(float2*, int, hipStream_t);

template <typename T>
void launch_local_grad(const C2<T>* X, const C2<T>* Y, int chiA, int chiC, double2* out,
                       hipStream_t st) {
    hipLaunchKernelGGL((k_local_grad<T>), dim3(256), dim3(256), 0, st, X, Y, chiA, chiC, out);
}
template void launch_local_grad<double>(const double2*, const double2*, int, int, double2*, hipStream_t);
template void launch_local_grad<float>(const float2*, const float2*, int, int, double2*, hipStream_t);

template <typename T>
void launch_transfer_left(const C2<T>* A, int chiL, int chiR, const double2* env_in,
                          const double2* v, double2* env_out, hipStream_t st) {
    hipLaunchKernelGGL((k_transfer_left<T>), dim3(chiR), dim3(256), 0, st, A, chiL, chiR, env_in, v,
                       env_out);
}

constexpr int kRightChunks = 64;

template <typename T>
void launch_transfer_right(const C2<T>* A, int chiL, int chiR, const double2* env_in,
                           const double2* v, double2* env_out, double2* scratch, hipStream_t st) {
    const int total = 4 * chiR;
    int chunks = total < kRightChunks ? total : kRightChunks;
    const int per = (total + chunks - 1) / chunks;
    chunks = (total + per - 1) / per;
    hipLaunchKernelGGL((k_transfer_right_part<T>), dim3((chiL + 255) / 256, chunks), dim3(256), 0, st,
                       A, chiL, chiR, env_in, v, per, scratch);
    hipLaunchKernelGGL(k_sum_chunks, dim3((chiL + 255) / 256), dim3(256), 0, st, scratch, chiL, chunks,
                       env_out);
}

void launch_dot(const double2* x, const double2* y, int len, double2* out, hipStream_t st) {
    hipLaunchKernelGGL(k_dot, dim3(1), dim3(256), 0, st, x, y, len, out);
}

// A[a, I, c] <- A[a, I, c] * fl(a) * fr(c) with fl = lamL[a] (or 1 / lamL[a]
// when invL), fr likewise; a null vector leaves that index alone.  The
// diagonal factors of the Gamma-lambda form (Sec. III.A, App. A).
template <typename T>
__global__ __launch_bounds__(256) void k_scale_site(C2<T>* __restrict__ A, int chiL, int chiR,
                                                    const double* __restrict__ lamL,
                                                    const double* __restrict__ lamR, int invL, int invR) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t total = (size_t)chiL * 4 * chiR;
    if (e >= total) return;
    const int a = (int)(e % chiL);
    const int c = (int)(e / (4 * (size_t)chiL));
    double f = 1.0;
    if (lamL) f = invL ? f / lamL[a] : f * lamL[a];
    if (lamR) f = invR ? f / lamR[c] : f * lamR[c];
    C2<T> v = A[e];
    v.x = (T)(v.x * f);
    v.y = (T)(v.y * f);
    A[e] = v;
}

template <typename T>
void launch_scale_site(C2<T>* A, int chiL, int chiR, const double* lamL, const double* lamR, bool invL,
                       bool invR, hipStream_t st) {
    const size_t total = (size_t)chiL * 4 * chiR;
    hipLaunchKernelGGL((k_scale_site<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, A, chiL,
                       chiR, lamL, lamR, invL ? 1 : 0, invR ? 1 : 0);
}
template void launch_scale_site<double>(double2*, int, int, const double*, const double*, bool, bool,
                                        hipStream_t);
template void launch_scale_site<float>(float2*, int, int, const double*, const double*, bool, bool,
                                       hipStream_t);

template void launch_transfer_left<double>(const double2*, int, int, const double2*, const double2*,
                                           double2*, hipStream_t);
template void launch_transfer_left<float>(const float2*, int, int, const double2*, const double2*,
                                          double2*, hipStream_t);
template void launch_transfer_right<double>(const double2*, int, int, const double2*,
                                            const double2*, double2*, double2*, hipStream_t);
template void launch_transfer_right<float>(const float2*, int, int, const double2*, const double2*,
                                           double2*, double2*, hipStream_t);

}  // namespace mpo

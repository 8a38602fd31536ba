// Per-kernel timing with HIP events on the launching stream (instrumentation).
// When enabled, each instrumented launch gets a start and a stop event (the
// Jacobi kernels through hipExtLaunchKernel, which stamps them with the
// dispatch's own start and end; the others bracketed by event records) and its
// algorithmic flop and byte counts are accumulated; elapsed times are
// collected lazily when the caller reads the statistics.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

namespace mpo {

enum KernelId {
    K_THETA = 0,     // two-site contraction + channel
    K_GRAM,          // Jacobi pair Gram
    K_EIG,           // Jacobi 64x64 FP64 eigen core
    K_UPDATE,        // Jacobi pair rotation
    K_NORMSORT,      // column norms + sort
    K_TRUNC,         // truncation weights + entropy
    K_GATHER,        // isometry gathers / transposes / copies
    K_GEMM,          // plain complex GEMMs (right factor, centre moves)
    K_TRANSFER,      // transfer contraction
    K_HGRAM,         // Gram matrix of the eigen-solver start
    K_TRIDIAG,       // tridiagonalisation: trailing Hermitian matrix-vector product (tiles)
    K_TRDAUX,        // tridiagonalisation: per-column step kernel, column norms, panel updates
    K_DC,            // divide and conquer on the tridiagonal
    K_BACK,          // back-transformation: reflector block products X Y, X -= P Y^H
    K_BTAUX,         // back-transformation: reflector mask, S = Y^H Y, P T, FP64 copy of X
    K_HOUT,          // X Q_H times the tridiagonal's eigenvectors (real GEMM)
    K_QR,            // Cholesky QR centre moves
    K_COUNT
};

inline const char* kernel_name(int k) {
    static const char* names[K_COUNT] = {"theta_channel", "jacobi_gram", "jacobi_eig64",
                                         "jacobi_update", "norm_sort",    "truncate",
                                         "gather",        "cgemm",        "transfer",
                                         "heev_gram",     "heev_trd_hemv", "heev_trd_step", "heev_dc",
                                         "heev_back",     "heev_bt_aux",   "heev_out",      "qr_move"};
    return names[k];
}

struct Profiler {
    struct Pending { hipEvent_t a, b; int k; };
    bool on = false;
    std::vector<hipEvent_t> free_events;
    std::vector<Pending> pending;
    long long launches[K_COUNT] = {};
    double ms[K_COUNT] = {};
    double flops[K_COUNT] = {};
    double bytes[K_COUNT] = {};
    hipEvent_t cur_a = nullptr;

    hipEvent_t get() {
        if (!free_events.empty()) { hipEvent_t e = free_events.back(); free_events.pop_back(); return e; }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    void begin(hipStream_t st) {
        if (!on) return;
        cur_a = get();
        (void)hipEventRecord(cur_a, st);
    }
    void end(hipStream_t st, int k, double fl, double by) {
        if (!on) return;
        hipEvent_t b = get();
        (void)hipEventRecord(b, st);
        pending.push_back({cur_a, b, k});
        launches[k] += 1;
        flops[k] += fl;
        bytes[k] += by;
        if (pending.size() >= 16384) collect();
    }
    // Events for hipExtLaunchKernel to stamp with the launch's own start and
    // stop (no separate event packets around it); both null when off.
    void stamps(hipEvent_t& a, hipEvent_t& b) {
        if (!on) { a = b = nullptr; return; }
        a = get();
        b = get();
    }
    void record(int k, hipEvent_t a, hipEvent_t b, double fl, double by) {
        if (!on) return;
        pending.push_back({a, b, k});
        launches[k] += 1;
        flops[k] += fl;
        bytes[k] += by;
        if (pending.size() >= 16384) collect();
    }
    // account work without a launch of its own (e.g. known only after a sweep)
    void add_work(int k, double fl, double by) {
        if (!on) return;
        flops[k] += fl;
        bytes[k] += by;
    }
    void collect() {
        if (pending.empty()) return;
        (void)hipEventSynchronize(pending.back().b);
        for (const Pending& p : pending) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) ms[p.k] += t;
            free_events.push_back(p.a);
            free_events.push_back(p.b);
        }
        pending.clear();
    }
    void reset() {
        collect();
        for (int k = 0; k < K_COUNT; ++k) { launches[k] = 0; ms[k] = flops[k] = bytes[k] = 0.0; }
    }
    ~Profiler() {
        collect();
        for (hipEvent_t e : free_events) (void)hipEventDestroy(e);
    }
};

}  // namespace mpo

// Batched evolution of independent circuits: host worker threads, one per
// caller stream, each owning an equal slice of the caller's arena.  A worker
// builds a handle for the circuit it takes (largest remaining first), runs the
// brickwork on its stream and writes the last-time-step observables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mpo.h"

// records an error message for the calling thread (defined in capi.hip)
void mpo_internal_set_error(const char* msg);

namespace {

size_t gates_of(int n, int depth) {
    return (size_t)((depth + 1) / 2) * (n / 2) + (size_t)(depth / 2) * (n / 2 - 1);
}

mpo_status slice_bytes(const mpo_batch_desc* c, int count, mpo_precision prec, size_t* out) {
    size_t mx = 0;
    for (int i = 0; i < count; ++i) {
        size_t b = 0;
        mpo_status st = mpo_workspace_bytes(c[i].n, c[i].chi_max, prec, &b);
        if (st != MPO_OK) return st;
        mx = std::max(mx, b);
    }
    *out = (mx + 255) & ~size_t(255);
    return MPO_OK;
}

}  // namespace

extern "C" mpo_status mpo_batch_workspace_bytes(const mpo_batch_desc* circuits, int count,
                                                mpo_precision prec, int n_streams, size_t* bytes) {
    if (!circuits || count < 1 || n_streams < 1 || !bytes) return MPO_ERR_ARG;
    size_t s = 0;
    mpo_status st = slice_bytes(circuits, count, prec, &s);
    if (st != MPO_OK) return st;
    *bytes = s * (size_t)n_streams;
    return MPO_OK;
}

extern "C" int mpo_batch_result_doubles(int n, int depth, int record_mask) {
    const int rows = ((record_mask & 1) && depth > 0) ? depth : 1;
    return rows * 2 * n + 2;
}

extern "C" mpo_status mpo_batch_run(const mpo_batch_desc* circuits, int count,
                                    const double* superops_concat, size_t n_superops,
                                    mpo_precision prec, mpo_basis basis, void* dev_arena,
                                    size_t arena_bytes, void* const* hip_streams, int n_streams,
                                    int use_graph, int record_mask, double* results) {
    if (!circuits || count < 1 || !superops_concat || !dev_arena || !results || n_streams < 1 ||
        !hip_streams)
        return MPO_ERR_ARG;
    if (use_graph)
        for (int w = 0; w < n_streams; ++w)
            if (!hip_streams[w]) {
                mpo_internal_set_error("use_graph needs non-null streams (a capture cannot use the null stream)");
                return MPO_ERR_ARG;
            }
    if (record_mask != 0 && record_mask != 1 && record_mask != 2) {
        mpo_internal_set_error("record_mask must be 0 or 2 (last time step) or 1 (every time step)");
        return MPO_ERR_ARG;
    }
    for (int i = 0; i < count; ++i) {
        const mpo_batch_desc& c = circuits[i];
        if (c.n < 2 || (c.n & 1) || c.depth < 0 || c.chi_max < 1 || c.chi_max > 1024 ||
            !(c.cutoff >= 0.0) || c.gate_offset + gates_of(c.n, c.depth) > n_superops)
            return MPO_ERR_ARG;
    }
    size_t slice = 0;
    mpo_status st = slice_bytes(circuits, count, prec, &slice);
    if (st != MPO_OK) return st;
    if (((uintptr_t)dev_arena) & 255) return MPO_ERR_ARG;
    if (arena_bytes < slice * (size_t)n_streams) return MPO_ERR_ARENA;

    // largest work first
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    auto work = [&](int i) {
        const mpo_batch_desc& c = circuits[i];
        return (double)c.n * c.depth * std::pow((double)c.chi_max, 3.0);
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });

    int device = 0;
    (void)hipGetDevice(&device);
    std::atomic<int> next{0};
    std::atomic<int> first_error{MPO_OK};
    std::vector<std::string> errs(n_streams);
    auto worker = [&](int w) {
        (void)hipSetDevice(device);
        char* base = (char*)dev_arena + slice * (size_t)w;
        for (;;) {
            const int k = next.fetch_add(1);
            if (k >= count || first_error.load() != MPO_OK) return;
            const mpo_batch_desc& c = circuits[order[k]];
            mpo_handle* h = nullptr;
            mpo_status s = mpo_create(c.n, c.chi_max, prec, basis, base, slice, hip_streams[w], &h);
            if (s == MPO_OK && use_graph) s = mpo_set_graphs(h, 1);
            if (s == MPO_OK) {
                const int g = (int)gates_of(c.n, c.depth);
                std::vector<double> disc((size_t)std::max(g, 1));
                double* out = results + c.result_offset;
                // rows recorded: every time step (record_mask 1) or the last one
                const bool every = (record_mask & 1) && c.depth > 0;
                const int rows = every ? c.depth : 1;
                double* S = out;
                double* Z = out + (size_t)rows * (c.n - 1);
                double* tr = Z + (size_t)rows * c.n;
                s = run_brickwork(h, c.depth, superops_concat + 512 * c.gate_offset, g, c.chi_max,
                                  c.cutoff, MPO_ORDER_ASCENDING, every ? 1 : 2, S, Z, tr, disc.data());
                if (s == MPO_OK) {
                    double tot = 0.0;
                    for (int q = 0; q < g; ++q) tot += disc[q];
                    tr[rows] = tot;
                    std::vector<int> dims(c.n - 1);
                    mpo_bond_dims(h, dims.data(), nullptr);
                    tr[rows + 1] = dims.empty() ? 1.0 : (double)*std::max_element(dims.begin(), dims.end());
                    if (c.depth == 0) {   // nothing recorded: product state values
                        for (int b = 0; b < c.n - 1; ++b) S[b] = 0.0;
                        s = mpo_expect_z_all(h, Z, tr);
                    }
                }
                if (s != MPO_OK) errs[w] = mpo_last_error();
                mpo_destroy(h);
            } else {
                errs[w] = mpo_last_error();
            }
            if (s != MPO_OK) {
                int expected = MPO_OK;
                first_error.compare_exchange_strong(expected, (int)s);
                return;
            }
        }
    };
    std::vector<std::thread> threads;
    for (int w = 1; w < n_streams; ++w) threads.emplace_back(worker, w);
    worker(0);
    for (auto& t : threads) t.join();
    for (int w = 0; w < n_streams; ++w)
        if (hip_streams[w]) (void)hipStreamSynchronize((hipStream_t)hip_streams[w]);
    if (first_error.load() != MPO_OK) {
        for (const std::string& e : errs)
            if (!e.empty()) { mpo_internal_set_error(e.c_str()); break; }
    }
    return (mpo_status)first_error.load();
}

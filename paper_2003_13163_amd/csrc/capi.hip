// libmpo C ABI: handle, arena layout and the host sequencing of the kernels.
//
// State: the vectorised density matrix (Sec. III.A) as an MPS with physical
// dimension 4 in mixed canonical form; site s holds A[a, I, c] at
// a + chiL*(I + 4c) in its own arena slot.  A gate follows the "Note added"
// update: exact centre moves, then contraction + channel + truncated SVD of the
// two-site block (App. A truncation).  Bond dimensions live on the host; the
// kept count of every split is read back once per split.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mpo.h"
#include "common.h"

using namespace mpo;

namespace {

thread_local std::string g_err;

mpo_status fail(mpo_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
mpo_status fail(mpo_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

struct HipError {
    hipError_t e;
    const char* what;
};

#define HIPCHK(x)                                              \
    do {                                                       \
        hipError_t _e = (x);                                   \
        if (_e != hipSuccess) throw HipError{_e, #x};          \
    } while (0)

struct NumericError { const char* what; };
struct NoConvError { const char* what; };
struct ArenaError { const char* what; };   // the handle's scratch cannot hold the request

constexpr int kMaxSuper = 1024;     // superoperators resident per upload
constexpr int64_t kMagicAny = 0x4d504f31;        // "MPO1": tensors in any gauge
constexpr int64_t kMagicCanonical = 0x4d504f32;  // "MPO2": mixed canonical about the stored centre
constexpr int kSplitsMax = 16;
constexpr int kMaxSweeps = 60;
constexpr int kRightChunksMax = 64;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Column stride of the SVD work matrices X, X2 with m rows: m + 8 (rounded up
// to even) complex values.  A power-of-two stride (m = 4 chi) puts the columns
// that one MFMA operand load touches into the same L1 cache sets.
inline int work_ld(int m) { return ((m + 1) & ~1) + 8; }

// Splits of at least this many columns start from the eigenvectors of the
// Gram matrix (heev.hip) when the handle's bond cap allows them; the eigen
// workspace is reserved for handles whose widest split, 4 chi_cap columns,
// reaches kHeevMinCols.
constexpr int kHeevMinCols = 512;
constexpr int kPrecondMinDefault = 1024;
// centre moves on bonds of at least this dimension use the Cholesky QR re-gauge
constexpr int kQrMinDefault = 128;

struct Layout {
    size_t slot_bytes, slots, x_bytes, r_bytes, partial_bytes, w_bytes, skip_bytes, vecN_bytes,
        info_bytes, env_bytes, tscr_bytes, vec_bytes, dot_bytes, super_bytes, heev_bytes, total;
    int max_pairs;
};

Layout make_layout(int n, int chi_cap, mpo_precision prec) {
    Layout L{};
    const size_t csz = prec == MPO_FP64 ? 16 : 8;
    const size_t cc = (size_t)chi_cap * chi_cap;
    L.slot_bytes = align256(4 * cc * csz);
    L.slots = (size_t)n + 2;
    L.x_bytes = align256((size_t)work_ld(4 * chi_cap) * 4 * chi_cap * csz);
    L.r_bytes = align256(cc * csz);
    int nb = (4 * chi_cap + 31) / 32;
    if (nb < 2) nb = 2;
    if (nb & 1) ++nb;
    L.max_pairs = nb / 2;
    L.partial_bytes = align256((size_t)L.max_pairs * kSplitsMax * 4096 * sizeof(double2));
    L.w_bytes = align256((size_t)L.max_pairs * 4096 * csz);
    L.skip_bytes = align256((size_t)4 * L.max_pairs * sizeof(int));   // 16-column blocks: 2x pairs
    L.vecN_bytes = align256((size_t)4 * chi_cap * sizeof(double));
    L.info_bytes = align256(sizeof(DevInfo));
    L.env_bytes = align256((size_t)(n + 1) * chi_cap * sizeof(double2));
    L.tscr_bytes = align256((size_t)kRightChunksMax * chi_cap * sizeof(double2));
    L.vec_bytes = align256((size_t)(n + 2) * 4 * sizeof(double2));
    L.dot_bytes = align256((size_t)(n + 2) * sizeof(double2));
    L.super_bytes = align256((size_t)kMaxSuper * 256 * csz);
    L.heev_bytes = 4 * chi_cap >= kHeevMinCols ? align256(heev_bytes(4 * chi_cap, 4 * chi_cap)) : 0;
    L.total = L.slot_bytes * L.slots + 2 * L.x_bytes + L.r_bytes + L.partial_bytes + L.w_bytes +
              L.skip_bytes + 3 * L.vecN_bytes + 2 * align256((size_t)chi_cap * sizeof(double)) +
              L.info_bytes + 2 * L.env_bytes + L.tscr_bytes +
              align256((size_t)chi_cap * sizeof(double2)) + L.vec_bytes + L.dot_bytes +
              L.super_bytes + L.heev_bytes;
    return L;
}

}  // namespace

void tuned_jacobi(mpo_precision prec, int chi_cap, int* block, int* inner);

struct mpo_handle {
    int n = 0, chi_cap = 0;
    mpo_precision prec = MPO_FP64;
    mpo_basis basis = MPO_BASIS_PAULI;
    hipStream_t st = nullptr;
    size_t csz = 16;
    bool bf3 = false;            // split-BF16x3 products on FP32 storage
    std::vector<char*> slot;     // slot base addresses
    std::vector<int> site_slot;  // slot index of every site
    std::vector<int> spare;      // free slot indices
    std::vector<int> dims;       // bond b in [0, n-2]
    int centre = 0;
    int qr_min = 0;              // centre moves by Cholesky QR on bonds of at least this size (0 = SVD moves)
    long long n_qr_fallback = 0; // QR moves that met rank deficiency and moved by the SVD instead
    bool poisoned = false;
    char *X = nullptr, *X2 = nullptr, *R = nullptr, *Mdev = nullptr;
    size_t x_bytes = 0;          // bytes of X and of X2 each
    JacobiWork jw{};
    HeevWork hw{};
    double2 *envL = nullptr, *envR = nullptr, *tscr = nullptr, *tmp = nullptr, *vecs = nullptr,
            *dots = nullptr;
    double* sig2_all = nullptr;  // copy of the last split's sorted squared values
    double *lamA = nullptr, *lamB = nullptr;   // lambda vectors of the Gamma-lambda update
    // pinned host staging
    DevInfo* info_host = nullptr;
    void* super_stage = nullptr;
    double2* small_host = nullptr;   // >= n+2 values
    double* sig_host = nullptr;      // 4*chi_cap
    Profiler prof;
    std::vector<double> last_S;      // per bond, filled by sweeps
    std::vector<std::vector<double>> last_lam;

    int chiL(int s) const { return s == 0 ? 1 : dims[s - 1]; }
    int chiR(int s) const { return s == n - 1 ? 1 : dims[s]; }
    char* site(int s) const { return slot[site_slot[s]]; }
    int take_spare() { int k = spare.back(); spare.pop_back(); return k; }
    void give_spare(int k) { spare.push_back(k); }
};

namespace {

double eps_of(size_t csz) { return csz == 16 ? 2.220446049250313e-16 : 1.1920928955078125e-07; }

// Convergence threshold on |g_ij| / sqrt(g_ii g_jj).  FP64: a few units of
// the Gram rounding sqrt(m) eps.  FP32: the Gram slabs are summed in FP64, so
// the off-diagonal noise is about eps32 * sqrt(slab) / sqrt(slabs); 2e-6 keeps
// the isometries orthonormal well below the 1e-4 entropy target.
// Split-BF16x3: every product term carries a relative error up to about
// 2^-15, so the off-diagonal measure has noise up to about 3e-5; 1e-4 is
// reachable and keeps the rotations' own error (2^-16 per update) below it.
// Those sweeps are followed by FP32-MFMA Gram sweeps down to kTolFp32.
double jacobi_tol(const mpo_handle* h, int m) {
    if (h->csz == 16) return std::fmax(1e-14, 8.0 * std::sqrt((double)m) * eps_of(h->csz));
    return h->bf3 ? 1e-4 : kTolFp32;
}
// singular values at or below this fraction of ||lambda||_2 carry no weight
// above rounding and are dropped by exact re-gauging moves
double regauge_cut(const mpo_handle* h) {
    if (h->bf3) return std::sqrt(kZeroRel2Bf3);
    return h->csz == 16 ? 1e-15 : std::sqrt(jacobi_zero_rel2<float>());
}

// Site dual vectors v[J] = Tr[P B_J] for the basis operators B_J.
void dual_vector(mpo_basis basis, int code, double2 v[4]) {
    for (int k = 0; k < 4; ++k) v[k] = make_double2(0.0, 0.0);
    if (basis == MPO_BASIS_PAULI) {
        v[code] = make_double2(std::sqrt(2.0), 0.0);
        return;
    }
    // computational: B_{2i+i'} = |i><i'|, Tr[P |i><i'|] = P[i'][i]
    switch (code) {
        case 0: v[0] = make_double2(1, 0); v[3] = make_double2(1, 0); break;
        case 1: v[1] = make_double2(1, 0); v[2] = make_double2(1, 0); break;
        case 2: v[1] = make_double2(0, 1); v[2] = make_double2(0, -1); break;
        case 3: v[0] = make_double2(1, 0); v[3] = make_double2(-1, 0); break;
    }
}

// Coefficients of |x><x| in the site basis.
void product_site(mpo_basis basis, int bit, double v[8]) {
    for (int k = 0; k < 8; ++k) v[k] = 0.0;
    if (basis == MPO_BASIS_COMPUTATIONAL) {
        v[2 * (3 * bit)] = 1.0;
    } else {
        const double s = 1.0 / std::sqrt(2.0);
        v[0] = s;                      // I component
        v[2 * 3] = bit ? -s : s;       // Z component
    }
}

// Scratch of the transfer contraction (FP64 environments, vectors, dot results).
struct ObsScratch {
    double2 *envL, *envR, *tscr, *tmp, *vecs, *dots;
};

template <typename T>
struct Engine {
    using C = C2<T>;
    static C* site(mpo_handle* h, int s) { return (C*)h->site(s); }

    static DevInfo read_info(mpo_handle* h) {
        HIPCHK(hipMemcpyAsync(h->info_host, h->jw.info, sizeof(DevInfo), hipMemcpyDeviceToHost, h->st));
        HIPCHK(hipStreamSynchronize(h->st));
        return *h->info_host;
    }

    // Orthogonalise the columns of X (m x N); truncation with (chi_max, cutoff).
    static DevInfo split(mpo_handle* h, int m, int N, int chi_max, double cutoff) {
        const int sw = jacobi_orthogonalize<T>((C*)h->X, m, N, work_ld(m), jacobi_tol(h, m), kMaxSweeps,
                                               h->jw, h->st, chi_max);
        if (sw == -2) HIPCHK(hipGetLastError());
        if (sw == -3) throw HipError{hipErrorInvalidValue, "jacobi pair capacity"};
        if (sw < 0) throw NoConvError{"one-sided Jacobi SVD did not converge"};
        // the decomposition may have kept only the leading columns (their
        // complement's weight is in the device info)
        const int n_out = h->jw.n_cols;
        h->prof.begin(h->st);
        launch_truncate(h->jw.sig2, n_out, chi_max, cutoff,
                        h->bf3 ? kZeroRel2Bf3 : jacobi_zero_rel2<T>(), h->jw.info, h->st, h->jw.rest_on);
        h->prof.end(h->st, K_TRUNC, 0.0, 8.0 * n_out);
        HIPCHK(hipGetLastError());
        DevInfo inf = read_info(h);
        if (inf.numeric_error) throw NumericError{"non-finite singular values"};
        return inf;
    }

    // The first r sorted singular values of the last split, to the host.
    static void read_values(mpo_handle* h, int r, std::vector<double>& lam) {
        HIPCHK(hipMemcpyAsync(h->sig_host, h->jw.sig2, sizeof(double) * r, hipMemcpyDeviceToHost, h->st));
        HIPCHK(hipStreamSynchronize(h->st));
        lam.resize(r);
        for (int i = 0; i < r; ++i) lam[i] = std::sqrt(std::fmax(h->sig_host[i], 0.0));
    }

    // Centre c -> c+1: L(A_c) = U R exactly; A_c <- U, A_{c+1} <- R A_{c+1}.
    // keep_values stores the singular values found (Schmidt values of bond c
    // when sites right of c+1 are right isometries) in last_lam[c]; cut < 0 is
    // the mode's re-gauge cut.
    static void move_right(mpo_handle* h, int c, bool keep_values = false, double cut = -1.0) {
        const int chiL = h->chiL(c), chiR = h->dims[c], chiR2 = h->chiR(c + 1);
        const int m = 4 * chiL, N = chiR;
        h->prof.begin(h->st);
        launch_copy_cols<T>(site(h, c), m, N, m, (C*)h->X, work_ld(m), h->st);
        h->prof.end(h->st, K_GATHER, 0.0, 2.0 * sizeof(C) * m * N);
        DevInfo inf = split(h, m, N, N, cut < 0.0 ? regauge_cut(h) : cut);
        const int r = inf.kept;
        if (keep_values) read_values(h, r, h->last_lam[c]);
        const int s1 = h->take_spare(), s2 = h->take_spare();
        C* U = (C*)h->slot[s1];
        C* Anext = (C*)h->slot[s2];
        h->prof.begin(h->st);
        launch_gather_cols<T>((C*)h->X, m, work_ld(m), h->jw.colmap, h->jw.sig2, r, U, m, h->st);
        h->prof.end(h->st, K_GATHER, 0.0, 2.0 * sizeof(C) * m * r);
        h->prof.begin(h->st);
        launch_cgemm<T>(1, 0, r, chiR, m, U, m, site(h, c), m, (C*)h->R, r, h->st, h->bf3);
        launch_cgemm<T>(0, 0, r, 4 * chiR2, chiR, (C*)h->R, r, site(h, c + 1), chiR, Anext, r, h->st, h->bf3);
        h->prof.end(h->st, K_GEMM, 8.0 * r * chiR * m + 8.0 * r * 4.0 * chiR2 * chiR,
                    (double)sizeof(C) * (2.0 * m * chiR + (double)m * r + 8.0 * chiR * chiR2 + 4.0 * r * chiR2));
        HIPCHK(hipGetLastError());
        h->give_spare(h->site_slot[c]);
        h->give_spare(h->site_slot[c + 1]);
        h->site_slot[c] = s1;
        h->site_slot[c + 1] = s2;
        h->dims[c] = r;
        h->centre = c + 1;
    }

    // Centre c -> c-1: R(A_c) = L Q exactly; the singular values found on the
    // way are the Schmidt values of bond c-1 (all other sites are isometries).
    static DevInfo move_left(mpo_handle* h, int c, bool keep_values, double cut = -1.0) {
        const int chiL = h->dims[c - 1], chiR = h->chiR(c), chiLL = h->chiL(c - 1);
        const int m = 4 * chiR, N = chiL;
        h->prof.begin(h->st);
        launch_conj_transpose<T>(site(h, c), chiL, m, chiL, (C*)h->X, work_ld(m), h->st);
        h->prof.end(h->st, K_GATHER, 0.0, 2.0 * sizeof(C) * m * chiL);
        DevInfo inf = split(h, m, N, N, cut < 0.0 ? regauge_cut(h) : cut);
        const int r = inf.kept;
        if (keep_values) read_values(h, r, h->last_lam[c - 1]);
        h->last_S[c - 1] = inf.entropy;
        const int s1 = h->take_spare(), s2 = h->take_spare();
        C* Q = (C*)h->slot[s1];
        C* Aprev = (C*)h->slot[s2];
        h->prof.begin(h->st);
        launch_gather_rows_conj<T>((C*)h->X, m, work_ld(m), h->jw.colmap, h->jw.sig2, r, Q, h->st);
        h->prof.end(h->st, K_GATHER, 0.0, 2.0 * sizeof(C) * m * r);
        h->prof.begin(h->st);
        launch_cgemm<T>(0, 1, chiL, r, m, site(h, c), chiL, Q, r, (C*)h->R, chiL, h->st, h->bf3);
        launch_cgemm<T>(0, 0, 4 * chiLL, r, chiL, site(h, c - 1), 4 * chiLL, (C*)h->R, chiL, Aprev,
                        4 * chiLL, h->st, h->bf3);
        h->prof.end(h->st, K_GEMM, 8.0 * chiL * r * m + 8.0 * 4.0 * chiLL * r * chiL,
                    (double)sizeof(C) * ((double)chiL * m + (double)r * m + 8.0 * chiLL * chiL + 4.0 * chiLL * r));
        HIPCHK(hipGetLastError());
        h->give_spare(h->site_slot[c]);
        h->give_spare(h->site_slot[c - 1]);
        h->site_slot[c] = s1;
        h->site_slot[c - 1] = s2;
        h->dims[c - 1] = r;
        h->centre = c - 1;
        return inf;
    }

    // Centre c -> c+1 by an exact QR of L(A_c) ("Note added"): A_c <- Q,
    // A_{c+1} <- R A_{c+1}; the bond keeps its dimension (no values dropped).
    // Returns false, with the state untouched, when L(A_c) is numerically
    // rank-deficient (the caller then moves by the SVD, which drops the null part).
    static bool move_right_qr(mpo_handle* h, int c) {
        const int chiL = h->chiL(c), r = h->dims[c], chiR2 = h->chiR(c + 1);
        const int m = 4 * chiL;
        const int s1 = h->take_spare(), s2 = h->take_spare();
        C* Q = (C*)h->slot[s1];
        C* Anext = (C*)h->slot[s2];
        if (!cholqr3<T>(site(h, c), m, r, m, Q, m, (C*)h->R, h->jw.info, h->info_host, h->hw, h->prof, h->st)) {
            h->give_spare(s2);
            h->give_spare(s1);
            h->n_qr_fallback += 1;
            return false;
        }
        h->prof.begin(h->st);
        launch_cgemm<T>(0, 0, r, 4 * chiR2, r, (C*)h->R, r, site(h, c + 1), r, Anext, r, h->st, h->bf3);
        h->prof.end(h->st, K_GEMM, 8.0 * r * 4.0 * chiR2 * r, (double)sizeof(C) * ((double)r * r + 8.0 * r * chiR2));
        HIPCHK(hipGetLastError());
        h->give_spare(h->site_slot[c]);
        h->give_spare(h->site_slot[c + 1]);
        h->site_slot[c] = s1;
        h->site_slot[c + 1] = s2;
        h->centre = c + 1;
        return true;
    }

    // Centre c -> c-1: R(A_c)^H = Q R, so R(A_c) = R^H Q^H; A_c <- Q^H,
    // A_{c-1} <- L(A_{c-1}) R^H.  False (state untouched) on rank deficiency.
    static bool move_left_qr(mpo_handle* h, int c) {
        const int r = h->dims[c - 1], chiR = h->chiR(c), chiLL = h->chiL(c - 1);
        const int m = 4 * chiR;
        h->prof.begin(h->st);
        launch_conj_transpose<T>(site(h, c), r, m, r, (C*)h->X, work_ld(m), h->st);
        h->prof.end(h->st, K_GATHER, 0.0, 2.0 * sizeof(C) * m * r);
        if (!cholqr3<T>((const C*)h->X, m, r, work_ld(m), (C*)h->X, work_ld(m), (C*)h->R, h->jw.info, h->info_host,
                        h->hw, h->prof, h->st)) {
            h->n_qr_fallback += 1;
            return false;
        }
        const int s1 = h->take_spare(), s2 = h->take_spare();
        C* Qh = (C*)h->slot[s1];
        C* Aprev = (C*)h->slot[s2];
        h->prof.begin(h->st);
        launch_conj_transpose<T>((C*)h->X, m, r, work_ld(m), Qh, r, h->st);
        launch_cgemm<T>(0, 1, 4 * chiLL, r, r, site(h, c - 1), 4 * chiLL, (C*)h->R, r, Aprev, 4 * chiLL, h->st,
                        h->bf3);
        h->prof.end(h->st, K_GEMM, 8.0 * 4.0 * chiLL * r * r, (double)sizeof(C) * (2.0 * m * r + 8.0 * chiLL * r + (double)r * r));
        HIPCHK(hipGetLastError());
        h->give_spare(h->site_slot[c]);
        h->give_spare(h->site_slot[c - 1]);
        h->site_slot[c] = s1;
        h->site_slot[c - 1] = s2;
        h->centre = c - 1;
        return true;
    }

    // Centre moves of the gate path: exact QR re-gauges where the handle has the
    // FP64 workspace, the bond is at least qr_min and the matrix to factor has at
    // least as many rows (4 x the outer bond) as columns; else the SVD moves.
    static bool use_qr(const mpo_handle* h, int bond_dim, int outer_dim) {
        return h->jw.heev && h->qr_min > 0 && bond_dim >= h->qr_min && 4 * outer_dim >= bond_dim;
    }
    static void move_centre(mpo_handle* h, int target) {
        while (h->centre < target) {
            const int c = h->centre;
            if (!(use_qr(h, h->dims[c], h->chiL(c)) && move_right_qr(h, c))) move_right(h, c);
        }
        while (h->centre > target) {
            const int c = h->centre;
            if (!(use_qr(h, h->dims[c - 1], h->chiR(c)) && move_left_qr(h, c))) move_left(h, c, false);
        }
    }

    // Gate on (s, s+1) with superoperator already on the device at Mg.
    static mpo_trunc_info apply(mpo_handle* h, int s, const C* Mg, int chi_max, double cutoff) {
        move_centre(h, s);
        const int chiL = h->chiL(s), chiM = h->dims[s], chiR = h->chiR(s + 1);
        const int m = 4 * chiL, N = 4 * chiR;
        h->prof.begin(h->st);
        launch_theta_channel<T>(chiL, chiM, chiR, site(h, s), site(h, s + 1), Mg, (C*)h->X,
                                (C*)h->X2, work_ld(m), h->st, h->bf3);
        h->prof.end(h->st, K_THETA, 8.0 * m * chiM * N + 2048.0 * chiL * chiR,
                    (double)sizeof(C) * (4.0 * chiL * chiM + 4.0 * chiM * chiR + 2.0 * m * N));
        HIPCHK(hipGetLastError());
        DevInfo inf = split(h, m, N, chi_max, cutoff);
        const int k = inf.kept;
        // A_s <- U_k (left isometry, in place); A_{s+1} <- U_k^H theta' (new centre)
        h->prof.begin(h->st);
        launch_gather_cols<T>((C*)h->X, m, work_ld(m), h->jw.colmap, h->jw.sig2, k, site(h, s), m, h->st);
        h->prof.end(h->st, K_GATHER, 0.0, 2.0 * sizeof(C) * m * k);
        h->prof.begin(h->st);
        launch_cgemm<T>(1, 0, k, N, m, site(h, s), m, (C*)h->X2, work_ld(m), site(h, s + 1), k, h->st,
                        h->bf3);
        h->prof.end(h->st, K_GEMM, 8.0 * k * N * m, (double)sizeof(C) * ((double)m * k + (double)m * N + (double)k * N));
        HIPCHK(hipGetLastError());
        h->dims[s] = k;
        h->centre = s + 1;
        mpo_trunc_info out;
        out.kept = k;
        out.discarded_weight = inf.discarded;
        out.total_weight = inf.total;
        out.entropy = inf.entropy;
        return out;
    }

    // The same gate with the split mirrored, for a sweep that moves left: the
    // centre comes to s+1, the rows of theta' are orthogonalised (Jacobi on
    // theta'^H), A_{s+1} <- V_k^H (right isometry) and A_s <- theta' V_k (new
    // centre, no division by a singular value).  The truncated state is the
    // same Schmidt truncation at bond s as in apply.
    static mpo_trunc_info apply_leftward(mpo_handle* h, int s, const C* Mg, int chi_max, double cutoff) {
        move_centre(h, s + 1);
        const int chiL = h->chiL(s), chiM = h->dims[s], chiR = h->chiR(s + 1);
        const int m = 4 * chiL, N = 4 * chiR;
        h->prof.begin(h->st);
        launch_theta_channel<T>(chiL, chiM, chiR, site(h, s), site(h, s + 1), Mg, (C*)h->X2, nullptr,
                                work_ld(m), h->st, h->bf3);
        h->prof.end(h->st, K_THETA, 8.0 * m * chiM * N + 2048.0 * chiL * chiR,
                    (double)sizeof(C) * (4.0 * chiL * chiM + 4.0 * chiM * chiR + 2.0 * m * N));
        h->prof.begin(h->st);
        launch_conj_transpose<T>((C*)h->X2, m, N, work_ld(m), (C*)h->X, work_ld(N), h->st);
        h->prof.end(h->st, K_GATHER, 0.0, 2.0 * sizeof(C) * m * N);
        HIPCHK(hipGetLastError());
        DevInfo inf = split(h, N, m, chi_max, cutoff);
        const int k = inf.kept;
        h->prof.begin(h->st);
        launch_gather_rows_conj<T>((C*)h->X, N, work_ld(N), h->jw.colmap, h->jw.sig2, k, site(h, s + 1),
                                   h->st);
        h->prof.end(h->st, K_GATHER, 0.0, 2.0 * sizeof(C) * N * k);
        h->prof.begin(h->st);
        launch_cgemm<T>(0, 1, m, k, N, (C*)h->X2, work_ld(m), site(h, s + 1), k, site(h, s), m, h->st,
                        h->bf3);
        h->prof.end(h->st, K_GEMM, 8.0 * m * k * N, (double)sizeof(C) * ((double)m * N + (double)k * N + (double)m * k));
        HIPCHK(hipGetLastError());
        h->dims[s] = k;
        h->centre = s;
        mpo_trunc_info out;
        out.kept = k;
        out.discarded_weight = inf.discarded;
        out.total_weight = inf.total;
        out.entropy = inf.entropy;
        return out;
    }

    // ------------------------------------------------ the paper's own update
    // App. A: the state in the Gamma-lambda form (Sec. III.A), a noisy gate on
    // the block B = lambda Gamma lambda Gamma lambda, its truncated SVD, then SVD
    // sweeps that restore the canonical form of the whole chain, every Gamma
    // recovered by dividing by the new lambda (Gamma <- W / lambda').  n - 1
    // decompositions per gate: O(n chi^3) per gate, against the local update's
    // O(chi^3) (the "Note added").  Sites hold the Gammas; lam[b] the lambdas.
    static void upload_lam(mpo_handle* h, const std::vector<double>& v, double* dst) {
        std::copy(v.begin(), v.end(), h->sig_host);   // pinned staging, reused: wait below
        HIPCHK(hipMemcpyAsync(dst, h->sig_host, sizeof(double) * v.size(), hipMemcpyHostToDevice, h->st));
        HIPCHK(hipStreamSynchronize(h->st));
    }

    static double vidal_gate(mpo_handle* h, int s, const C* Mg, int chi_max, double cutoff, double drop,
                             std::vector<std::vector<double>>& lam) {
        const int n = h->n;
        const int chiL = h->chiL(s), chiM = h->dims[s], chiR = h->chiR(s + 1);
        const int m = 4 * chiL, N = 4 * chiR;
        // B = lambda_{s-1} Gamma_s lambda_s Gamma_{s+1} lambda_{s+1} (scalings applied in place)
        if (s > 0) upload_lam(h, lam[s - 1], h->lamA);
        upload_lam(h, lam[s], h->lamB);
        launch_scale_site<T>(site(h, s), chiL, chiM, s > 0 ? h->lamA : nullptr, h->lamB, false, false, h->st);
        if (s + 1 < n - 1) {
            upload_lam(h, lam[s + 1], h->lamA);
            launch_scale_site<T>(site(h, s + 1), chiM, chiR, nullptr, h->lamA, false, false, h->st);
        }
        launch_theta_channel<T>(chiL, chiM, chiR, site(h, s), site(h, s + 1), Mg, (C*)h->X, (C*)h->X2,
                                work_ld(m), h->st, h->bf3);
        HIPCHK(hipGetLastError());
        DevInfo inf = split(h, m, N, chi_max, cutoff);
        std::vector<double> lp;
        read_values(h, inf.kept, lp);
        // Gamma = W / lambda' is undefined for lambda' = 0: values at or below
        // drop * lambda'_max are removed before any division
        int k = 0;
        while (k < (int)lp.size() && lp[k] > drop * lp[0]) ++k;
        k = std::max(1, k);
        lp.resize(k);
        // site s <- U lambda' (the columns as they are), site s+1 <- U^H theta' = lambda' V^H
        const int su = h->take_spare();
        C* U = (C*)h->slot[su];
        launch_gather_cols<T>((C*)h->X, m, work_ld(m), h->jw.colmap, h->jw.sig2, k, U, m, h->st, true);
        launch_cgemm<T>(1, 0, k, N, m, U, m, (C*)h->X2, work_ld(m), site(h, s + 1), k, h->st, h->bf3);
        launch_gather_cols<T>((C*)h->X, m, work_ld(m), h->jw.colmap, h->jw.sig2, k, site(h, s), m, h->st,
                              false);
        HIPCHK(hipGetLastError());
        h->give_spare(su);
        h->dims[s] = k;
        lam[s] = lp;
        // left sweep (B_<-): bonds s-1 .. 0
        std::vector<double> cur = lp;
        for (int j = s; j >= 1; --j) {
            if (j - 1 >= 1) {   // site j-1 <- lambda_{j-2} Gamma_{j-1}
                upload_lam(h, lam[j - 2], h->lamA);
                launch_scale_site<T>(site(h, j - 1), h->chiL(j - 1), h->dims[j - 1], h->lamA, nullptr, false,
                                     false, h->st);
            }
            h->centre = j;
            move_left(h, j, true, drop);            // site j <- W, site j-1 <- site j-1 . (V L)
            upload_lam(h, cur, h->lamB);            // Gamma_j = W / lambda_j
            launch_scale_site<T>(site(h, j), h->dims[j - 1], h->chiR(j), nullptr, h->lamB, false, true, h->st);
            lam[j - 1] = h->last_lam[j - 1];
            cur = lam[j - 1];
        }
        // site 0 ends as Gamma_0 lambda_0 (the last move multiplied it by V L):
        // Gamma_0 = site 0 / lambda_0; for s = 0 it holds U lambda', Gamma_0 = U
        upload_lam(h, s == 0 ? lp : lam[0], h->lamB);
        launch_scale_site<T>(site(h, 0), 1, h->dims[0], nullptr, h->lamB, false, true, h->st);
        // right sweep (B_->): bonds s+1 .. n-2
        cur = lp;
        for (int j = s + 1; j <= n - 2; ++j) {
            if (j + 1 <= n - 2) {   // site j+1 <- Gamma_{j+1} lambda_{j+1}
                upload_lam(h, lam[j + 1], h->lamA);
                launch_scale_site<T>(site(h, j + 1), h->dims[j], h->chiR(j + 1), nullptr, h->lamA, false, false,
                                     h->st);
            }
            h->centre = j;
            move_right(h, j, true, drop);           // site j <- Q, site j+1 <- (L W) . site j+1
            upload_lam(h, cur, h->lamB);            // Gamma_j = Q / lambda_{j-1}
            launch_scale_site<T>(site(h, j), h->dims[j - 1], h->dims[j], h->lamB, nullptr, true, false, h->st);
            lam[j] = h->last_lam[j];
            cur = lam[j];
        }
        // site n-1 ends as lambda_{n-2} Gamma_{n-1} (the last move multiplied it
        // by L W): Gamma_{n-1} = site n-1 / lambda_{n-2}; for s + 1 = n - 1 it
        // holds lambda' V^H, Gamma_{n-1} = V^H
        upload_lam(h, s + 1 == n - 1 ? lp : lam[n - 2], h->lamB);
        launch_scale_site<T>(site(h, n - 1), h->dims[n - 2], 1, h->lamB, nullptr, true, false, h->st);
        HIPCHK(hipGetLastError());
        return inf.discarded;
    }

    static double entropy_of(const std::vector<double>& l) {
        double tot = 0.0, S = 0.0;
        for (double v : l) tot += v * v;
        if (tot <= 0.0) return 0.0;
        for (double v : l) {
            const double w = v * v / tot;
            if (w > 0.0) S -= w * std::log2(w);
        }
        return S;
    }

    static void run_vidal(mpo_handle* h, int depth, const double* superops, int n_gates, int chi_max,
                          double cutoff, double* S_out, double* discarded_out) {
        const int n = h->n;
        constexpr double drop = 1e-14;
        init_product(h, nullptr);                    // Gamma = |0><0| site vectors, lambda = (1)
        std::vector<std::vector<double>> lam(n - 1, std::vector<double>(1, 1.0));
        int g = 0, resident0 = 0, resident = 0;
        for (int t = 0; t < depth; ++t) {
            for (int s = (t % 2 == 0) ? 0 : 1; s + 1 < n; s += 2, ++g) {
                if (g >= resident0 + resident) {
                    resident0 = g;
                    resident = std::min(kMaxSuper, n_gates - g);
                    HIPCHK(hipStreamSynchronize(h->st));
                    upload_super(h, superops + (size_t)g * 512, resident);
                }
                const double d = vidal_gate(h, s, (const C*)h->Mdev + (size_t)(g - resident0) * 256, chi_max,
                                            cutoff, drop, lam);
                if (discarded_out) discarded_out[g] = d;
            }
            if (S_out)
                for (int b = 0; b < n - 1; ++b) S_out[(size_t)t * (n - 1) + b] = entropy_of(lam[b]);
        }
        // back to the mixed canonical form: A_s = lambda_{s-1} Gamma_s (left
        // isometries), the centre at n-1
        for (int s = 1; s < n; ++s) {
            upload_lam(h, lam[s - 1], h->lamA);
            launch_scale_site<T>(site(h, s), h->chiL(s), h->chiR(s), h->lamA, nullptr, false, false, h->st);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(h->st));
        h->centre = n - 1;
    }

    static void upload_super(mpo_handle* h, const double* superops, int count) {
        T* stage = (T*)h->super_stage;
        for (size_t i = 0; i < (size_t)count * 512; ++i) stage[i] = (T)superops[i];
        HIPCHK(hipMemcpyAsync(h->Mdev, stage, (size_t)count * 256 * sizeof(C), hipMemcpyHostToDevice, h->st));
    }

    // Canonical sweep: centre to n-1, then to 0, recording every bond.
    static void sweep_all(mpo_handle* h, bool keep_values) {
        move_centre(h, h->n - 1);
        for (int c = h->n - 1; c > 0; --c) move_left(h, c, keep_values);
    }

    // Tr rho and all <Z_i> numerators by transfer contraction (Sec. III.D).
    static void observables(mpo_handle* h, double* z, double* trace_re, double* trace_im) {
        observables_in(h, ObsScratch{h->envL, h->envR, h->tscr, h->tmp, h->vecs, h->dots}, z, trace_re,
                       trace_im);
    }
    // The same contraction with its environments in the given scratch.
    static void observables_in(mpo_handle* h, const ObsScratch& w, double* z, double* trace_re,
                               double* trace_im) {
        const int n = h->n, cap = h->chi_cap;
        double2 *const envL = w.envL, *const envR = w.envR, *const tscr = w.tscr, *const tmp = w.tmp,
                       *const vecs = w.vecs, *const dots = w.dots;
        double2 hv[8];
        dual_vector(h->basis, 0, hv);
        dual_vector(h->basis, 3, hv + 4);
        HIPCHK(hipMemcpyAsync(vecs, hv, sizeof(hv), hipMemcpyHostToDevice, h->st));
        const double2 one = make_double2(1.0, 0.0);
        HIPCHK(hipMemcpyAsync(envL, &one, sizeof(one), hipMemcpyHostToDevice, h->st));
        HIPCHK(hipMemcpyAsync(envR + (size_t)n * cap, &one, sizeof(one), hipMemcpyHostToDevice, h->st));
        for (int s = 0; s < n; ++s)
            launch_transfer_left<T>(site(h, s), h->chiL(s), h->chiR(s), envL + (size_t)s * cap,
                                    vecs, envL + (size_t)(s + 1) * cap, h->st);
        if (z) {
            for (int s = n - 1; s >= 0; --s)
                launch_transfer_right<T>(site(h, s), h->chiL(s), h->chiR(s),
                                         envR + (size_t)(s + 1) * cap, vecs,
                                         envR + (size_t)s * cap, tscr, h->st);
            for (int i = 0; i < n; ++i) {
                launch_transfer_left<T>(site(h, i), h->chiL(i), h->chiR(i), envL + (size_t)i * cap,
                                        vecs + 4, tmp, h->st);
                launch_dot(tmp, envR + (size_t)(i + 1) * cap, h->chiR(i), dots + i, h->st);
            }
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(h->small_host, envL + (size_t)n * cap, sizeof(double2),
                              hipMemcpyDeviceToHost, h->st));
        if (z)
            HIPCHK(hipMemcpyAsync(h->small_host + 1, dots, sizeof(double2) * n,
                                  hipMemcpyDeviceToHost, h->st));
        HIPCHK(hipStreamSynchronize(h->st));
        const double2 tr = h->small_host[0];
        if (trace_re) *trace_re = tr.x;
        if (trace_im) *trace_im = tr.y;
        if (z) {
            const double den = tr.x * tr.x + tr.y * tr.y;
            for (int i = 0; i < n; ++i) {
                const double2 v = h->small_host[1 + i];
                z[i] = (v.x * tr.x + v.y * tr.y) / den;   // Re(v / tr)
            }
        }
    }

    static void pauli(mpo_handle* h, const unsigned char* codes, double* re, double* im) {
        const int n = h->n, cap = h->chi_cap;
        std::vector<double2> hv((size_t)(n + 1) * 4);
        for (int s = 0; s < n; ++s) dual_vector(h->basis, codes[s], &hv[(size_t)4 * s]);
        dual_vector(h->basis, 0, &hv[(size_t)4 * n]);
        HIPCHK(hipMemcpyAsync(h->vecs, hv.data(), sizeof(double2) * hv.size(), hipMemcpyHostToDevice, h->st));
        const double2 one = make_double2(1.0, 0.0);
        HIPCHK(hipMemcpyAsync(h->envL, &one, sizeof(one), hipMemcpyHostToDevice, h->st));
        HIPCHK(hipMemcpyAsync(h->envR, &one, sizeof(one), hipMemcpyHostToDevice, h->st));
        for (int s = 0; s < n; ++s) {
            launch_transfer_left<T>(site(h, s), h->chiL(s), h->chiR(s), h->envL + (size_t)s * cap,
                                    h->vecs + 4 * s, h->envL + (size_t)(s + 1) * cap, h->st);
            launch_transfer_left<T>(site(h, s), h->chiL(s), h->chiR(s), h->envR + (size_t)s * cap,
                                    h->vecs + 4 * n, h->envR + (size_t)(s + 1) * cap, h->st);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(h->small_host, h->envL + (size_t)n * cap, sizeof(double2), hipMemcpyDeviceToHost, h->st));
        HIPCHK(hipMemcpyAsync(h->small_host + 1, h->envR + (size_t)n * cap, sizeof(double2), hipMemcpyDeviceToHost, h->st));
        HIPCHK(hipStreamSynchronize(h->st));
        const double2 num = h->small_host[0], tr = h->small_host[1];
        const double den = tr.x * tr.x + tr.y * tr.y;
        *re = (num.x * tr.x + num.y * tr.y) / den;
        *im = (num.y * tr.x - num.x * tr.y) / den;
    }

    // Site vectors of the projectors |0><0| = (1 + Z)/2 and |1><1| = (1 - Z)/2.
    static void projector_vectors(mpo_basis basis, double2 v[8]) {
        double2 vi[4], vz[4];
        dual_vector(basis, 0, vi);
        dual_vector(basis, 3, vz);
        for (int k = 0; k < 4; ++k) {
            v[k] = make_double2(0.5 * (vi[k].x + vz[k].x), 0.5 * (vi[k].y + vz[k].y));
            v[4 + k] = make_double2(0.5 * (vi[k].x - vz[k].x), 0.5 * (vi[k].y - vz[k].y));
        }
    }

    // P(x) = Tr[|x><x| rho] (Sec. III.D): one transfer step per site.
    static void probability(mpo_handle* h, const unsigned char* bits, double* re, double* im) {
        const int n = h->n, cap = h->chi_cap;
        std::vector<double2> hv((size_t)4 * n);
        double2 pv[8];
        projector_vectors(h->basis, pv);
        for (int s = 0; s < n; ++s)
            for (int k = 0; k < 4; ++k) hv[(size_t)4 * s + k] = pv[4 * bits[s] + k];
        HIPCHK(hipMemcpyAsync(h->vecs, hv.data(), sizeof(double2) * hv.size(), hipMemcpyHostToDevice, h->st));
        const double2 one = make_double2(1.0, 0.0);
        HIPCHK(hipMemcpyAsync(h->envL, &one, sizeof(one), hipMemcpyHostToDevice, h->st));
        for (int s = 0; s < n; ++s)
            launch_transfer_left<T>(site(h, s), h->chiL(s), h->chiR(s), h->envL + (size_t)s * cap,
                                    h->vecs + 4 * s, h->envL + (size_t)(s + 1) * cap, h->st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(h->small_host, h->envL + (size_t)n * cap, sizeof(double2), hipMemcpyDeviceToHost, h->st));
        HIPCHK(hipStreamSynchronize(h->st));
        *re = h->small_host[0].x;
        *im = h->small_host[0].y;
    }

    // Sequential conditional sampling (Sec. III.D).  The right environments
    // sum every later site out (identity vector); per site one GEMM forms the
    // prefix environments times the site tensor for all samples of a chunk,
    // and k_sample_site draws the dit.  Chunks are sized to the X / X2 scratch.
    static void sample(mpo_handle* h, int count, const double* uniforms, unsigned char* bits_out,
                       double* prob_out, int* clamped_out) {
        const int n = h->n, cap = h->chi_cap;
        int chimax = 1;
        for (int b = 0; b < n - 1; ++b) chimax = std::max(chimax, h->dims[b]);
        const size_t csz = sizeof(C);
        const size_t per2 = 2 * (size_t)chimax * csz + (size_t)n * 9 + 16;   // X2 bytes per sample
        const size_t avail2 = h->x_bytes > 2048 ? h->x_bytes - 2048 : 0;   // alignment slack
        size_t chunk = std::min(h->x_bytes / (4 * (size_t)chimax * csz), avail2 / per2);
        chunk = std::min(chunk, (size_t)count);
        if (chunk < 1) throw ArenaError{"the handle's scratch cannot hold one sample"};
        // right environments with the identity vector: envR[k] sums sites k..n-1 out
        double2 hv[12];
        dual_vector(h->basis, 0, hv);
        projector_vectors(h->basis, hv + 4);
        HIPCHK(hipMemcpyAsync(h->vecs, hv, sizeof(hv), hipMemcpyHostToDevice, h->st));
        const double2 one = make_double2(1.0, 0.0);
        HIPCHK(hipMemcpyAsync(h->envR + (size_t)n * cap, &one, sizeof(one), hipMemcpyHostToDevice, h->st));
        for (int s = n - 1; s >= 0; --s)
            launch_transfer_right<T>(site(h, s), h->chiL(s), h->chiR(s), h->envR + (size_t)(s + 1) * cap,
                                     h->vecs, h->envR + (size_t)s * cap, h->tscr, h->st);
        auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
        std::vector<C> last(chunk);
        std::vector<double> logn(chunk);
        std::vector<int> clam(chunk);
        int n_clamped = 0;
        for (size_t s0 = 0; s0 < (size_t)count; s0 += chunk) {
            const int S = (int)std::min(chunk, (size_t)count - s0);
            char* q = h->X2;
            C* La = (C*)q; q += al((size_t)chimax * S * csz);
            C* Lb = (C*)q; q += al((size_t)chimax * S * csz);
            double* u = (double*)q; q += al((size_t)S * n * 8);
            unsigned char* bits = (unsigned char*)q; q += al((size_t)S * n);
            double* logN = (double*)q; q += al((size_t)S * 8);
            int* clamped = (int*)q;
            C* Y = (C*)h->X;
            HIPCHK(hipMemcpyAsync(u, uniforms + s0 * n, (size_t)S * n * 8, hipMemcpyHostToDevice, h->st));
            launch_sample_init<T>(La, logN, clamped, S, h->st);
            for (int k = 0; k < n; ++k) {
                const int cl = h->chiL(k), cr = h->chiR(k);
                launch_cgemm<T>(1, 0, 4 * cr, S, cl, site(h, k), cl, La, cl, Y, 4 * cr, h->st, h->bf3);
                launch_sample_site<T>(Y, cr, S, h->envR + (size_t)(k + 1) * cap, h->vecs + 4, u, n, k,
                                      Lb, bits, logN, clamped, h->st);
                std::swap(La, Lb);
            }
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(bits_out + s0 * n, bits, (size_t)S * n, hipMemcpyDeviceToHost, h->st));
            HIPCHK(hipMemcpyAsync(last.data(), La, (size_t)S * csz, hipMemcpyDeviceToHost, h->st));
            HIPCHK(hipMemcpyAsync(logn.data(), logN, (size_t)S * 8, hipMemcpyDeviceToHost, h->st));
            HIPCHK(hipMemcpyAsync(clam.data(), clamped, (size_t)S * 4, hipMemcpyDeviceToHost, h->st));
            HIPCHK(hipStreamSynchronize(h->st));
            for (int i = 0; i < S; ++i) {
                if (prob_out) prob_out[s0 + i] = (double)last[i].x * std::exp(logn[i]);
                n_clamped += clam[i];
            }
        }
        if (clamped_out) *clamped_out = n_clamped;
    }

    static void init_product(mpo_handle* h, const unsigned char* bits) {
        for (int b = 0; b < h->n - 1; ++b) h->dims[b] = 1;
        std::vector<T> buf(8);
        for (int s = 0; s < h->n; ++s) {
            double v[8];
            product_site(h->basis, bits ? bits[s] : 0, v);
            for (int k = 0; k < 8; ++k) buf[k] = (T)v[k];
            HIPCHK(hipMemcpyAsync(site(h, s), buf.data(), sizeof(T) * 8, hipMemcpyHostToDevice, h->st));
            HIPCHK(hipStreamSynchronize(h->st));
        }
        h->centre = 0;
    }

    static size_t export_size(const mpo_handle* h) {
        size_t bytes = (size_t)(4 + h->n - 1) * 8;
        for (int s = 0; s < h->n; ++s) bytes += (size_t)h->chiL(s) * 4 * h->chiR(s) * 16;
        return bytes;
    }

    static void do_export(mpo_handle* h, char* out) {
        int64_t* hdr = (int64_t*)out;
        hdr[0] = kMagicCanonical;
        hdr[1] = h->n;
        hdr[2] = h->basis;
        hdr[3] = h->centre;
        for (int b = 0; b < h->n - 1; ++b) hdr[4 + b] = h->dims[b];
        double* dst = (double*)(out + (size_t)(4 + h->n - 1) * 8);
        std::vector<C> tmp;
        for (int s = 0; s < h->n; ++s) {
            const int cl = h->chiL(s), cr = h->chiR(s);
            tmp.resize((size_t)cl * 4 * cr);
            HIPCHK(hipMemcpyAsync(tmp.data(), site(h, s), sizeof(C) * tmp.size(), hipMemcpyDeviceToHost, h->st));
            HIPCHK(hipStreamSynchronize(h->st));
            for (int a = 0; a < cl; ++a)
                for (int I = 0; I < 4; ++I)
                    for (int c = 0; c < cr; ++c) {
                        const C v = tmp[(size_t)a + (size_t)cl * (I + 4 * c)];
                        const size_t o = ((size_t)(a * 4 + I) * cr + c) * 2;
                        dst[o] = (double)v.x;
                        dst[o + 1] = (double)v.y;
                    }
            dst += (size_t)cl * 4 * cr * 2;
        }
    }

    static void do_import(mpo_handle* h, const char* in) {
        const int64_t* hdr = (const int64_t*)in;
        for (int b = 0; b < h->n - 1; ++b) h->dims[b] = (int)hdr[4 + b];
        const double* src = (const double*)(in + (size_t)(4 + h->n - 1) * 8);
        std::vector<C> tmp;
        for (int s = 0; s < h->n; ++s) {
            const int cl = h->chiL(s), cr = h->chiR(s);
            tmp.resize((size_t)cl * 4 * cr);
            for (int a = 0; a < cl; ++a)
                for (int I = 0; I < 4; ++I)
                    for (int c = 0; c < cr; ++c) {
                        const size_t o = ((size_t)(a * 4 + I) * cr + c) * 2;
                        C v;
                        v.x = (T)src[o];
                        v.y = (T)src[o + 1];
                        tmp[(size_t)a + (size_t)cl * (I + 4 * c)] = v;
                    }
            HIPCHK(hipMemcpyAsync(site(h, s), tmp.data(), sizeof(C) * tmp.size(), hipMemcpyHostToDevice, h->st));
            HIPCHK(hipStreamSynchronize(h->st));
            src += (size_t)cl * 4 * cr * 2;
        }
        if (hdr[0] == kMagicCanonical) {
            // written by mpo_export: already in mixed canonical form about hdr[3]
            h->centre = (int)hdr[3];
        } else {
            // any gauge: a left-to-right sweep of exact QR-type moves canonicalises
            h->centre = 0;
            move_centre(h, h->n - 1);
        }
    }
};

// ----------------------------------------------------------------- adjoint
// Frozen-projector gradient of O = sum_i Tr[Z_i rho_D].  With the kept
// subspace of every truncation frozen, gate g is the linear map
// rho -> P_g M_g rho, P_g = (Phi_g Phi_g^H) (x) 1 with Phi_g the left isometries
// of sites 0..s after the gate; moves are exact identities.  The co-state
// mu_G = w, lambda_g = P_g mu_g, mu_{g-1} = M_g^H lambda_g is carried as an MPS
// of its own; dO/dM_g = <lambda_g | E_(IJ,KL) rho_{g-1}> is a two-site contraction.
// In an ascending layer, after the projection at its last gate the co-state's
// sites left of every earlier gate of the layer already are that gate's frozen
// isometries, so only one projection (an environment sweep) per layer is
// needed, and the left overlap of lambda_g with rho_{g-1} is the identity.
struct AdjLayout {
    size_t slot_bytes, tape_slots, ckpt_slots, mu_bytes, env_bytes, y_bytes, t1_bytes, th_bytes, mh_bytes,
        total;
    int chi_mu, seg;           // co-state bond cap; time steps per recomputed segment
};

// Slots per recorded time step: the n sites at its start, every pre-gate centre
// (at most n/2) and the sites 0..last after its last gate (at most n), plus one.
size_t adj_tape_slots_per_step(int n) { return 2 * (size_t)n + (size_t)n / 2 + 1; }

AdjLayout adj_layout(int n, int depth, int chi_max, mpo_precision prec, int n_gates, int checkpoint_every) {
    AdjLayout L{};
    const size_t csz = prec == MPO_FP64 ? 16 : 8;
    const size_t cm = (size_t)chi_max;
    L.chi_mu = std::min(1024, 4 * chi_max);
    L.seg = (checkpoint_every <= 0 || checkpoint_every > depth) ? depth : checkpoint_every;
    const size_t cu = (size_t)L.chi_mu;
    L.slot_bytes = align256(4 * cm * cm * csz);
    L.tape_slots = (size_t)L.seg * adj_tape_slots_per_step(n);
    // one state of n sites at the start of every segment, plus the final state
    L.ckpt_slots = ((size_t)(depth + L.seg - 1) / L.seg + 1) * (size_t)n;
    size_t mu = 0;
    mpo_workspace_bytes(n, L.chi_mu, prec, &mu);
    L.mu_bytes = align256(mu);
    L.env_bytes = align256(cm * cu * csz);
    L.y_bytes = align256(4 * std::max(cm, cu) * std::max(cm, cu) * csz);
    L.t1_bytes = align256(4 * cm * cu * csz);
    L.th_bytes = align256(16 * cm * cu * csz);
    L.mh_bytes = align256(((size_t)n_gates + 1) * 256 * csz);
    L.total = L.slot_bytes * (L.tape_slots + L.ckpt_slots) + L.mu_bytes + 4 * L.env_bytes + L.y_bytes +
              L.t1_bytes + 2 * L.th_bytes + L.mh_bytes + align256(256 * sizeof(double2));
    return L;
}

template <typename T>
struct Adjoint {
    using C = C2<T>;
    using E = Engine<T>;
    struct Tape {
        int first = 0, last = 0;
        std::vector<int> pre_dims;        // bonds 0..n-2 at the start of the layer
        std::vector<C*> pre;              // n site tensors (centre at `first`)
        std::vector<C*> cen;              // pre-gate centre tensor of every gate
        std::vector<int> cen_l, cen_r;    // its bond dimensions
        std::vector<C*> post;             // sites 0..last after the last gate
        std::vector<int> post_dims;       // bonds 0..last
    };

    static void copy_site(mpo_handle* h, int s, C* dst, int cl, int cr) {
        launch_copy<T>(E::site(h, s), dst, (size_t)cl * 4 * cr, h->st);
    }

    // S_q from S_{q+1}: S_q[c, c'] = sum conj(lam[c', I, d']) rho[c, I, d] S_{q+1}[d, d']
    static void right_step(mpo_handle* h, const C* rho, int rl, int rr, const C* lam, int ll, int lr,
                           const C* Sin, C* Sout, C* Y) {
        launch_cgemm<T>(0, 0, 4 * rl, lr, rr, rho, 4 * rl, Sin, rr, Y, 4 * rl, h->st, h->bf3);
        launch_cgemm<T>(0, 1, rl, ll, 4 * lr, Y, rl, lam, ll, Sout, rl, h->st, h->bf3);
    }
    // E_{q+1}[a', b'] = sum conj(phi[a, I, a']) E_q[a, b] mu[b, I, b']
    static void left_step(mpo_handle* h, const C* phi, int pl, int pr, const C* mu, int ml, int mr,
                          const C* Ein, C* Eout, C* Y) {
        launch_cgemm<T>(0, 0, pl, 4 * mr, ml, Ein, pl, mu, ml, Y, pl, h->st, h->bf3);
        launch_cgemm<T>(1, 0, pr, mr, 4 * pl, phi, 4 * pl, Y, 4 * pl, Eout, pr, h->st, h->bf3);
    }

    static void set_one(mpo_handle* h, C* dst) {
        C one;
        one.x = T(1);
        one.y = T(0);
        HIPCHK(hipMemcpyAsync(dst, &one, sizeof(C), hipMemcpyHostToDevice, h->st));
        HIPCHK(hipStreamSynchronize(h->st));
    }

    // mu <- w = sum_i (Z at i, identity elsewhere) as a bond-2 MPS
    static void init_observable(mpo_handle* mu) {
        const int n = mu->n;
        double2 t[4], z[4];
        dual_vector(mu->basis, 0, t);
        dual_vector(mu->basis, 3, z);
        for (int b = 0; b < n - 1; ++b) mu->dims[b] = 2;
        for (int s = 0; s < n; ++s) {
            const int cl = s == 0 ? 1 : 2, cr = s == n - 1 ? 1 : 2;
            std::vector<C> buf((size_t)cl * 4 * cr);
            for (auto& v : buf) { v.x = T(0); v.y = T(0); }
            auto put = [&](int a, int I, int c, double2 v) {
                C& e = buf[(size_t)a + (size_t)cl * (I + 4 * c)];
                e.x = (T)v.x;
                e.y = (T)(-v.y);   // w = conj(dual vector): <w|rho> = sum dual * rho
            };
            for (int I = 0; I < 4; ++I) {
                if (s == 0 && n > 1) { put(0, I, 0, t[I]); put(0, I, 1, z[I]); }
                else if (s == n - 1) { put(0, I, 0, z[I]); put(1, I, 0, t[I]); }
                else { put(0, I, 0, t[I]); put(0, I, 1, z[I]); put(1, I, 1, t[I]); }
            }
            HIPCHK(hipMemcpyAsync(E::site(mu, s), buf.data(), sizeof(C) * buf.size(), hipMemcpyHostToDevice, mu->st));
            HIPCHK(hipStreamSynchronize(mu->st));
        }
        mu->centre = 0;
    }

    static void run(mpo_handle* h, int depth, const double* superops, int n_gates, int chi_max,
                    double cutoff, char* work, const AdjLayout& L, double* O_out, double* grads,
                    int* costate_max_bond) {
        const int n = h->n;
        // ---- carve the workspace
        char* p = work;
        char* tape_base = p;
        p += L.slot_bytes * L.tape_slots;
        char* ckpt_base = p;
        p += L.slot_bytes * L.ckpt_slots;
        char* mu_arena = p; p += L.mu_bytes;
        C* env[4];
        for (int k = 0; k < 4; ++k) { env[k] = (C*)p; p += L.env_bytes; }
        C* Y = (C*)p; p += L.y_bytes;
        C* T1 = (C*)p; p += L.t1_bytes;
        C* THL = (C*)p; p += L.th_bytes;
        C* TH = (C*)p; p += L.th_bytes;
        C* MH = (C*)p; p += L.mh_bytes;
        double2* gdev = (double2*)p;
        // first gate of every time step
        std::vector<int> g_first(depth + 1, 0);
        for (int t = 0; t < depth; ++t) g_first[t + 1] = g_first[t] + ((t % 2 == 0) ? n / 2 : n / 2 - 1);
        // superoperators resident on the device, uploaded in windows of kMaxSuper gates
        int resident0 = 0, resident = 0;
        auto gate_ptr = [&](int g) -> const C* {
            if (g < resident0 || g >= resident0 + resident) {
                resident0 = g;
                resident = std::min(kMaxSuper, n_gates - g);
                HIPCHK(hipStreamSynchronize(h->st));   // the pinned staging buffer is reused
                E::upload_super(h, superops + (size_t)g * 512, resident);
            }
            return (const C*)h->Mdev + (size_t)(g - resident0) * 256;
        };
        // Checkpoint c holds the state at the start of time step c * seg, the last
        // one the final state.  The backward recomputes one segment of seg time
        // steps at a time from its checkpoint, recording the tape of that segment
        // only; the kernels are deterministic, so the recomputed steps repeat the
        // first forward bit for bit and the frozen projectors are the forward's.
        const int n_seg = (depth + L.seg - 1) / L.seg;
        std::vector<std::vector<int>> ck_dims(n_seg + 1);
        std::vector<int> ck_centre(n_seg + 1, 0);
        auto ck_site = [&](int c, int s) { return (C*)(ckpt_base + L.slot_bytes * ((size_t)c * n + s)); };
        auto save = [&](int c) {
            ck_dims[c] = h->dims;
            ck_centre[c] = h->centre;
            for (int s = 0; s < n; ++s) copy_site(h, s, ck_site(c, s), h->chiL(s), h->chiR(s));
        };
        auto restore = [&](int c) {
            h->dims = ck_dims[c];
            h->centre = ck_centre[c];
            for (int s = 0; s < n; ++s)
                launch_copy<T>(ck_site(c, s), E::site(h, s), (size_t)h->chiL(s) * 4 * h->chiR(s), h->st);
            HIPCHK(hipGetLastError());
        };
        size_t next_slot = 0;
        auto take = [&]() -> C* {
            if (next_slot >= L.tape_slots) throw HipError{hipErrorOutOfMemory, "adjoint tape"};
            return (C*)(tape_base + L.slot_bytes * next_slot++);
        };
        // One forward time step; with a tape, the state at its start, every
        // pre-gate centre and the left isometries after its last gate.  Both
        // forms make the same moves and launches in the same order.
        auto step = [&](int t, Tape* tp) {
            const int first = (t % 2 == 0) ? 0 : 1;
            int g = g_first[t];
            if (tp) {
                tp->first = first;
                E::move_centre(h, first);
                tp->pre_dims = h->dims;
                for (int s = 0; s < n; ++s) {
                    tp->pre.push_back(take());
                    copy_site(h, s, tp->pre.back(), h->chiL(s), h->chiR(s));
                }
            }
            for (int s = first; s + 1 < n; s += 2, ++g) {
                const C* Mg = gate_ptr(g);
                E::move_centre(h, s);
                if (tp) {
                    tp->cen.push_back(take());
                    tp->cen_l.push_back(h->chiL(s));
                    tp->cen_r.push_back(h->dims[s]);
                    copy_site(h, s, tp->cen.back(), h->chiL(s), h->dims[s]);
                }
                E::apply(h, s, Mg, chi_max, cutoff);
                if (tp) tp->last = s;
            }
            if (tp) {
                for (int s = 0; s <= tp->last; ++s) {
                    tp->post.push_back(take());
                    copy_site(h, s, tp->post.back(), h->chiL(s), h->chiR(s));
                }
                tp->post_dims.assign(h->dims.begin(), h->dims.begin() + tp->last + 1);
            }
        };
        // ---- forward, keeping only the checkpoints
        for (int t = 0; t < depth; ++t) {
            if (t % L.seg == 0) save(t / L.seg);
            step(t, nullptr);
        }
        save(n_seg);
        HIPCHK(hipGetLastError());
        {
            std::vector<double> z(n);
            double tr = 0.0;
            E::observables(h, z.data(), &tr, nullptr);
            double O = 0.0;
            for (int i = 0; i < n; ++i) O += z[i] * tr;
            *O_out = O;
        }
        // ---- co-state and adjoint superoperators
        mpo_handle* mu = nullptr;
        mpo_status cst = mpo_create(n, L.chi_mu, h->prec, h->basis, mu_arena, L.mu_bytes, h->st, &mu);
        if (cst != MPO_OK) throw HipError{hipErrorOutOfMemory, "co-state handle"};
        std::unique_ptr<mpo_handle, void (*)(mpo_handle*)> mu_guard(mu, mpo_destroy);
        init_observable(mu);
        {
            std::vector<T> mh((size_t)n_gates * 512 + 512);
            for (int q = 0; q < n_gates; ++q)
                for (int r = 0; r < 16; ++r)
                    for (int c = 0; c < 16; ++c) {   // (M^H)[r][c] = conj(M[c][r])
                        mh[(size_t)q * 512 + 2 * (16 * r + c)] = (T)superops[(size_t)q * 512 + 2 * (16 * c + r)];
                        mh[(size_t)q * 512 + 2 * (16 * r + c) + 1] = (T)(-superops[(size_t)q * 512 + 2 * (16 * c + r) + 1]);
                    }
            for (int r = 0; r < 16; ++r) mh[(size_t)n_gates * 512 + 2 * (16 * r + r)] = T(1);
            HIPCHK(hipMemcpyAsync(MH, mh.data(), sizeof(T) * mh.size(), hipMemcpyHostToDevice, h->st));
            HIPCHK(hipStreamSynchronize(h->st));
        }
        const C* Id = MH + (size_t)n_gates * 256;
        int co_max = 2;
        // ---- backward, one recomputed segment at a time
        std::vector<Tape> tape;
        int g = n_gates;
        for (int t = depth - 1; t >= 0; --t) {
            if (t == depth - 1 || (t + 1) % L.seg == 0) {
                const int c = t / L.seg, t0 = c * L.seg;
                restore(c);
                tape.assign(t - t0 + 1, Tape());
                next_slot = 0;
                for (int u = t0; u <= t; ++u) step(u, &tape[u - t0]);
                HIPCHK(hipGetLastError());
            }
            Tape& tp = tape[t % L.seg];
            const int m_gates = (int)tp.cen.size();
            const int sm = tp.last;
            auto pre_l = [&](int s) { return s == 0 ? 1 : tp.pre_dims[s - 1]; };
            auto pre_r = [&](int s) { return s == n - 1 ? 1 : tp.pre_dims[s]; };
            auto post_l = [&](int s) { return s == 0 ? 1 : tp.post_dims[s - 1]; };
            // (1) projection at the layer's last gate: sites 0..sm <- Phi, E into site sm+1
            C* Ea = env[0];
            C* Eb = env[1];
            set_one(h, Ea);
            for (int q = 0; q <= sm; ++q) {
                left_step(h, tp.post[q], post_l(q), tp.post_dims[q], E::site(mu, q), mu->chiL(q),
                          mu->chiR(q), Ea, Eb, Y);
                std::swap(Ea, Eb);
            }
            {
                const int k = tp.post_dims[sm], ml = mu->chiL(sm + 1), mr = mu->chiR(sm + 1);
                const int sl = mu->take_spare();
                launch_cgemm<T>(0, 0, k, 4 * mr, ml, Ea, k, E::site(mu, sm + 1), ml, (C*)mu->slot[sl], k, h->st, h->bf3);
                mu->give_spare(mu->site_slot[sm + 1]);
                mu->site_slot[sm + 1] = sl;
                for (int q = 0; q <= sm; ++q)
                    launch_copy<T>(tp.post[q], E::site(mu, q), (size_t)post_l(q) * 4 * tp.post_dims[q], h->st);
                for (int b = 0; b <= sm; ++b) mu->dims[b] = tp.post_dims[b];
            }
            // (2) right environment of the last gate: sites >= sm+2
            C* Sa = env[2];
            C* Sb = env[3];
            set_one(h, Sa);
            for (int q = n - 1; q >= sm + 2; --q) {
                right_step(h, tp.pre[q], pre_l(q), pre_r(q), E::site(mu, q), mu->chiL(q), mu->chiR(q), Sa, Sb, Y);
                std::swap(Sa, Sb);
            }
            // (3) gates of the layer, last to first
            for (int j = m_gates - 1; j >= 0; --j) {
                --g;
                const int s = tp.first + 2 * j;
                const int ca = mu->chiL(s), cb = mu->dims[s], cc = mu->chiR(s + 1);
                if (ca != tp.cen_l[j]) throw HipError{hipErrorInvalidValue, "adjoint bond mismatch"};
                // theta_lambda and Theta = theta_rho contracted with the right environment
                launch_theta_channel<T>(ca, cb, cc, E::site(mu, s), E::site(mu, s + 1), Id, THL, nullptr, 4 * ca,
                                        h->st, h->bf3);
                const int rs = tp.cen_r[j], rr = pre_r(s + 1);
                launch_cgemm<T>(0, 0, 4 * rs, cc, rr, tp.pre[s + 1], 4 * rs, Sa, rr, T1, 4 * rs, h->st, h->bf3);
                launch_cgemm<T>(0, 0, 4 * ca, 4 * cc, rs, tp.cen[j], 4 * ca, T1, rs, TH, 4 * ca, h->st, h->bf3);
                launch_local_grad<T>(THL, TH, ca, cc, gdev, h->st);
                HIPCHK(hipMemcpyAsync(grads + (size_t)g * 512, gdev, 256 * sizeof(double2), hipMemcpyDeviceToHost, h->st));
                // mu <- M^H lambda on (s, s+1).  The co-state needs no canonical
                // form, so when the bond fits it is split exactly as I * theta:
                // site s the identity on (I, a), site s+1 theta itself (bond 4 ca,
                // the generic rank).  Otherwise an SVD split capped at chi_mu.
                const int m = 4 * ca, N = 4 * cc;
                int r;
                if (m <= L.chi_mu) {
                    const int sl = mu->take_spare();
                    launch_theta_channel<T>(ca, cb, cc, E::site(mu, s), E::site(mu, s + 1),
                                            MH + (size_t)g * 256, (C*)mu->slot[sl], nullptr, m, h->st, h->bf3);
                    launch_identity_site<T>(E::site(mu, s), ca, h->st);
                    mu->give_spare(mu->site_slot[s + 1]);
                    mu->site_slot[s + 1] = sl;
                    r = m;
                } else {
                    launch_theta_channel<T>(ca, cb, cc, E::site(mu, s), E::site(mu, s + 1),
                                            MH + (size_t)g * 256, (C*)mu->X, (C*)mu->X2, work_ld(m), h->st,
                                            h->bf3);
                    HIPCHK(hipGetLastError());
                    DevInfo inf = E::split(mu, m, N, L.chi_mu, regauge_cut(mu));
                    r = inf.kept;
                    launch_gather_cols<T>((C*)mu->X, m, work_ld(m), mu->jw.colmap, mu->jw.sig2, r, E::site(mu, s), m,
                                          h->st);
                    launch_cgemm<T>(1, 0, r, N, m, E::site(mu, s), m, (C*)mu->X2, work_ld(m), E::site(mu, s + 1), r,
                                    h->st, h->bf3);
                }
                co_max = std::max(co_max, r);
                mu->dims[s] = r;
                // right environment for the previous gate of the layer: sites >= s
                if (j > 0) {
                    right_step(h, tp.pre[s + 1], pre_l(s + 1), pre_r(s + 1), E::site(mu, s + 1), r, cc, Sa, Sb, Y);
                    std::swap(Sa, Sb);
                    right_step(h, tp.pre[s], pre_l(s), pre_r(s), E::site(mu, s), mu->chiL(s), r, Sa, Sb, Y);
                    std::swap(Sa, Sb);
                }
                HIPCHK(hipGetLastError());
            }
        }
        restore(n_seg);
        HIPCHK(hipStreamSynchronize(h->st));
        if (costate_max_bond) *costate_max_bond = co_max;
    }
};

template <typename F>
mpo_status guarded(mpo_handle* h, F&& f) {
    try {
        f();
        return MPO_OK;
    } catch (const HipError& e) {
        return fail(MPO_ERR_HIP, "HIP error %s in %s", hipGetErrorString(e.e), e.what);
    } catch (const NumericError& e) {
        if (h) h->poisoned = true;
        return fail(MPO_ERR_NUMERIC, "%s", e.what);
    } catch (const NoConvError& e) {
        if (h) h->poisoned = true;
        return fail(MPO_ERR_NOCONV, "%s", e.what);
    } catch (const ArenaError& e) {
        return fail(MPO_ERR_ARENA, "%s", e.what);
    } catch (const HeevFailure& e) {
        return fail(MPO_ERR_HIP, "eigen-solver: %s", e.what);
    }
}

#define DISPATCH(h, ...)                                                 \
    do {                                                                 \
        if ((h)->prec == MPO_FP64) { using E = Engine<double>; __VA_ARGS__; } \
        else { using E = Engine<float>; __VA_ARGS__; }                   \
    } while (0)

mpo_status check_live(mpo_handle* h) {
    if (!h) return fail(MPO_ERR_ARG, "null handle");
    if (h->poisoned) return fail(MPO_ERR_STATE, "handle poisoned by an earlier numeric fault");
    return MPO_OK;
}

bool finite_all(const double* v, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

}  // namespace

// ------------------------------------------------- allocation-free scratch
// Device scratch for mpo_expect_z_all_noalloc: a file-scope device array, one
// copy per GPU, resident while the library is loaded.  Host code must never
// pass the array's own name to a kernel or a copy (on the host it is only a
// stand-in symbol): its device address is looked up once per device with
// hipGetSymbolAddress and that address is used everywhere.
constexpr size_t kStaticScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device); nullptr with the error message set on failure.
void* static_scratch() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        fail(MPO_ERR_HIP, "no current HIP device for the static scratch");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            fail(MPO_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_dev[dev] = ptr;
    }
    return g_scratch_dev[dev];
}

// Transfer-contraction scratch of an n-site handle with bond cap `cap`, carved
// from `base` (or only measured when base is null); returns the bytes used.
size_t carve_obs_scratch(char* base, int n, int cap, ObsScratch* w) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align256(bytes);
        return (double2*)p;
    };
    ObsScratch o;
    o.envL = take((size_t)(n + 1) * cap * sizeof(double2));
    o.envR = take((size_t)(n + 1) * cap * sizeof(double2));
    o.tscr = take((size_t)kRightChunksMax * cap * sizeof(double2));
    o.tmp = take((size_t)cap * sizeof(double2));
    o.vecs = take((size_t)(n + 2) * 4 * sizeof(double2));
    o.dots = take((size_t)(n + 2) * sizeof(double2));
    if (w) *w = o;
    return off;
}
}  // namespace

void mpo_internal_set_error(const char* msg) { g_err = msg ? msg : ""; }

// ------------------------------------------------------------ tuning table
// Jacobi block width and inner sweeps per precision and bond cap, filled by
// the autotuner (mpo_set_default_tuning); a handle picks the first entry of
// its precision whose chi_upto covers its chi_cap, else the built-in default.
namespace {
struct TuneEntry { int prec, chi_upto, block, inner; };
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;
}  // namespace

void tuned_jacobi(mpo_precision prec, int chi_cap, int* block, int* inner) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const TuneEntry* best = nullptr;
    for (const TuneEntry& e : g_tune)
        if (e.prec == (int)prec && e.chi_upto >= chi_cap && (!best || e.chi_upto < best->chi_upto)) best = &e;
    if (best) {
        *block = best->block;
        *inner = best->inner;
    }
}

// ==================================================================== C ABI
extern "C" {

const char* mpo_last_error(void) { return g_err.c_str(); }

mpo_status mpo_workspace_bytes(int n, int chi_cap, mpo_precision prec, size_t* bytes) {
    if (!bytes) return fail(MPO_ERR_ARG, "bytes is NULL");
    if (n < 2 || (n & 1)) return fail(MPO_ERR_ARG, "n must be even and >= 2 (got %d)", n);
    if (chi_cap < 1 || chi_cap > 1024) return fail(MPO_ERR_ARG, "chi_cap must be in [1, 1024] (got %d)", chi_cap);
    if (prec != MPO_FP64 && prec != MPO_FP32_MFMA && prec != MPO_BF16X3)
        return fail(MPO_ERR_ARG, "unknown precision %d", (int)prec);
    *bytes = make_layout(n, chi_cap, prec).total;
    return MPO_OK;
}

mpo_status mpo_create(int n, int chi_cap, mpo_precision prec, mpo_basis basis, void* dev_arena,
                      size_t arena_bytes, void* hip_stream, mpo_handle** out) {
    if (!out) return fail(MPO_ERR_ARG, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    mpo_status st = mpo_workspace_bytes(n, chi_cap, prec, &need);
    if (st != MPO_OK) return st;
    if (basis != MPO_BASIS_PAULI && basis != MPO_BASIS_COMPUTATIONAL)
        return fail(MPO_ERR_ARG, "unknown basis %d", (int)basis);
    if (!dev_arena) return fail(MPO_ERR_ARG, "dev_arena is NULL");
    if (((uintptr_t)dev_arena) & 255) return fail(MPO_ERR_ARG, "dev_arena must be 256-byte aligned");
    if (arena_bytes < need)
        return fail(MPO_ERR_ARENA, "arena has %zu bytes, %zu needed", arena_bytes, need);
    mpo_handle* h = new mpo_handle();
    h->n = n;
    h->chi_cap = chi_cap;
    h->prec = prec;
    h->basis = basis;
    h->st = (hipStream_t)hip_stream;
    h->csz = prec == MPO_FP64 ? 16 : 8;
    h->bf3 = prec == MPO_BF16X3;
    const Layout L = make_layout(n, chi_cap, prec);
    char* p = (char*)dev_arena;
    h->slot.resize(L.slots);
    for (size_t k = 0; k < L.slots; ++k) { h->slot[k] = p; p += L.slot_bytes; }
    h->site_slot.resize(n);
    for (int s = 0; s < n; ++s) h->site_slot[s] = s;
    h->spare = {n, n + 1};
    h->x_bytes = L.x_bytes;
    h->X = p; p += L.x_bytes;
    h->X2 = p; p += L.x_bytes;
    h->R = p; p += L.r_bytes;
    h->jw.gram_partials = p; p += L.partial_bytes;
    h->jw.w = p; p += L.w_bytes;
    h->jw.skip = (int*)p; p += L.skip_bytes;
    h->jw.nrm2 = (double*)p; p += L.vecN_bytes;
    h->jw.sig2 = (double*)p; p += L.vecN_bytes;
    h->jw.colmap = (int*)p; p += L.vecN_bytes;
    h->lamA = (double*)p; p += align256((size_t)chi_cap * sizeof(double));
    h->lamB = (double*)p; p += align256((size_t)chi_cap * sizeof(double));
    h->jw.info = (DevInfo*)p; p += L.info_bytes;
    h->jw.max_pairs = L.max_pairs;
    h->jw.splits = kSplitsMax;
    h->jw.prof = &h->prof;
    h->jw.bf3 = h->bf3;
    h->jw.block = 16;
    // one inner sweep per block pair is the faster setting wherever the outer
    // tolerance is loose (FP32, BF16x3); FP64 gains nothing from it
    h->jw.inner = prec == MPO_FP64 ? 2 : 1;
    tuned_jacobi(prec, chi_cap, &h->jw.block, &h->jw.inner);
    if (const char* e = std::getenv("MPO_JACOBI_BLOCK")) h->jw.block = std::atoi(e) == 16 ? 16 : 32;
    if (const char* e = std::getenv("MPO_JACOBI_INNER")) h->jw.inner = std::max(1, std::min(8, std::atoi(e)));
    h->jw.trace = std::getenv("MPO_JACOBI_TRACE") != nullptr;
    h->jw.graphs = false;
    h->jw.graph_cache = jacobi_graph_cache_new();
    h->envL = (double2*)p; p += L.env_bytes;
    h->envR = (double2*)p; p += L.env_bytes;
    h->tscr = (double2*)p; p += L.tscr_bytes;
    h->tmp = (double2*)p; p += align256((size_t)chi_cap * sizeof(double2));
    h->vecs = (double2*)p; p += L.vec_bytes;
    h->dots = (double2*)p; p += L.dot_bytes;
    h->Mdev = p; p += L.super_bytes;
    h->jw.heev = nullptr;
    h->jw.precond_min = 0;
    h->jw.n_precond = 0;
    h->jw.n_checks = 0;
    if (L.heev_bytes) {
        heev_carve(p, 4 * chi_cap, 4 * chi_cap, h->hw);
        p += L.heev_bytes;
        h->hw.plans = heev_plans_new();
        h->jw.heev = &h->hw;
        h->jw.precond_min = kPrecondMinDefault;
        if (const char* e = std::getenv("MPO_PRECOND_MIN")) h->jw.precond_min = std::max(0, std::atoi(e));
        h->qr_min = kQrMinDefault;
        if (const char* e = std::getenv("MPO_QR_MIN")) h->qr_min = std::max(0, std::atoi(e));
    }
    h->dims.assign(n - 1, 1);
    h->last_S.assign(n - 1, 0.0);
    h->last_lam.assign(n - 1, std::vector<double>());
    if (hipHostMalloc((void**)&h->info_host, sizeof(DevInfo)) != hipSuccess ||
        hipHostMalloc(&h->super_stage, (size_t)kMaxSuper * 256 * h->csz) != hipSuccess ||
        hipHostMalloc((void**)&h->small_host, sizeof(double2) * (n + 4)) != hipSuccess ||
        hipHostMalloc((void**)&h->sig_host, sizeof(double) * 4 * chi_cap) != hipSuccess) {
        mpo_destroy(h);
        return fail(MPO_ERR_HIP, "pinned host allocation failed");
    }
    h->jw.info_host = h->info_host;
    st = guarded(h, [&] { DISPATCH(h, E::init_product(h, nullptr)); });
    if (st != MPO_OK) { mpo_destroy(h); return st; }
    *out = h;
    return MPO_OK;
}

void mpo_destroy(mpo_handle* h) {
    if (!h) return;
    if (h->st) (void)hipStreamSynchronize(h->st); else (void)hipDeviceSynchronize();
    if (h->info_host) (void)hipHostFree(h->info_host);
    if (h->super_stage) (void)hipHostFree(h->super_stage);
    if (h->small_host) (void)hipHostFree(h->small_host);
    if (h->sig_host) (void)hipHostFree(h->sig_host);
    jacobi_graph_cache_free(h->jw.graph_cache);
    heev_plans_free(h->hw.plans);
    delete h;
}

mpo_status mpo_init_product(mpo_handle* h, const unsigned char* bits) {
    if (!h) return fail(MPO_ERR_ARG, "null handle");
    if (bits)
        for (int s = 0; s < h->n; ++s)
            if (bits[s] > 1) return fail(MPO_ERR_ARG, "bits[%d] = %d is not 0/1", s, bits[s]);
    mpo_status st = guarded(h, [&] { DISPATCH(h, E::init_product(h, bits)); });
    if (st == MPO_OK) h->poisoned = false;
    return st;
}

mpo_status mpo_apply_2q_channel(mpo_handle* h, int site, const double* superop, int chi_max,
                                double cutoff, mpo_trunc_info* info) {
    mpo_status st = check_live(h);
    if (st != MPO_OK) return st;
    if (site < 0 || site > h->n - 2) return fail(MPO_ERR_ARG, "site %d out of [0, %d]", site, h->n - 2);
    if (!superop) return fail(MPO_ERR_ARG, "superop is NULL");
    if (chi_max < 1 || chi_max > h->chi_cap)
        return fail(MPO_ERR_ARG, "chi_max %d out of [1, %d]", chi_max, h->chi_cap);
    if (!(cutoff >= 0.0) || !std::isfinite(cutoff)) return fail(MPO_ERR_ARG, "cutoff must be finite and >= 0");
    if (!finite_all(superop, 512)) {
        h->poisoned = true;
        return fail(MPO_ERR_NUMERIC, "non-finite superoperator entry");
    }
    return guarded(h, [&] {
        DISPATCH(h, {
            E::upload_super(h, superop, 1);
            mpo_trunc_info r = E::apply(h, site, (const typename E::C*)h->Mdev, chi_max, cutoff);
            if (info) *info = r;
        });
    });
}

mpo_status mpo_canonicalize(mpo_handle* h, int center) {
    mpo_status st = check_live(h);
    if (st != MPO_OK) return st;
    if (center < 0 || center >= h->n) return fail(MPO_ERR_ARG, "center %d out of range", center);
    return guarded(h, [&] { DISPATCH(h, E::move_centre(h, center)); });
}

mpo_status mpo_bond_entropy(mpo_handle* h, int bond, double* S) {
    mpo_status st = check_live(h);
    if (st != MPO_OK) return st;
    if (!S) return fail(MPO_ERR_ARG, "S is NULL");
    if (bond < -1 || bond > h->n - 2) return fail(MPO_ERR_ARG, "bond %d out of range", bond);
    return guarded(h, [&] {
        DISPATCH(h, {
            if (bond < 0) {
                E::sweep_all(h, false);
                for (int b = 0; b < h->n - 1; ++b) S[b] = h->last_S[b];
            } else {
                E::move_centre(h, bond + 1);
                E::move_left(h, bond + 1, false);
                *S = h->last_S[bond];
            }
        });
    });
}

mpo_status mpo_singular_values(mpo_handle* h, int bond, double* lam, int cap, int* count) {
    mpo_status st = check_live(h);
    if (st != MPO_OK) return st;
    if (bond < 0 || bond > h->n - 2) return fail(MPO_ERR_ARG, "bond %d out of range", bond);
    if (!count || (cap > 0 && !lam)) return fail(MPO_ERR_ARG, "null output");
    return guarded(h, [&] {
        DISPATCH(h, {
            E::move_centre(h, bond + 1);
            E::move_left(h, bond + 1, true);
            const std::vector<double>& v = h->last_lam[bond];
            *count = (int)v.size();
            for (int i = 0; i < cap && i < (int)v.size(); ++i) lam[i] = v[i];
        });
    });
}

mpo_status mpo_expect_pauli(mpo_handle* h, const unsigned char* pauli, double* re, double* im) {
    mpo_status st = check_live(h);
    if (st != MPO_OK) return st;
    if (!pauli || !re || !im) return fail(MPO_ERR_ARG, "null argument");
    for (int s = 0; s < h->n; ++s)
        if (pauli[s] > 3) return fail(MPO_ERR_ARG, "pauli[%d] = %d not in 0..3", s, pauli[s]);
    return guarded(h, [&] { DISPATCH(h, E::pauli(h, pauli, re, im)); });
}

mpo_status mpo_trace(mpo_handle* h, double* re, double* im) {
    mpo_status st = check_live(h);
    if (st != MPO_OK) return st;
    if (!re || !im) return fail(MPO_ERR_ARG, "null argument");
    return guarded(h, [&] { DISPATCH(h, E::observables(h, nullptr, re, im)); });
}

mpo_status mpo_probability(mpo_handle* h, const unsigned char* bits, double* re, double* im) {
    mpo_status st = check_live(h);
    if (st != MPO_OK) return st;
    if (!bits || !re || !im) return fail(MPO_ERR_ARG, "null argument");
    for (int s = 0; s < h->n; ++s)
        if (bits[s] > 1) return fail(MPO_ERR_ARG, "bits[%d] = %d is not 0/1", s, bits[s]);
    return guarded(h, [&] { DISPATCH(h, E::probability(h, bits, re, im)); });
}

mpo_status mpo_sample(mpo_handle* h, int n_samples, const double* uniforms, unsigned char* bits,
                      double* prob, int* clamped) {
    mpo_status st = check_live(h);
    if (st != MPO_OK) return st;
    if (n_samples < 1 || !uniforms || !bits) return fail(MPO_ERR_ARG, "bad sampling arguments");
    for (size_t i = 0; i < (size_t)n_samples * h->n; ++i)
        if (!(uniforms[i] >= 0.0 && uniforms[i] < 1.0))
            return fail(MPO_ERR_ARG, "uniforms[%zu] = %g is not in [0, 1)", i, uniforms[i]);
    return guarded(h, [&] { DISPATCH(h, E::sample(h, n_samples, uniforms, bits, prob, clamped)); });
}

mpo_status mpo_expect_z_all(mpo_handle* h, double* z, double* trace) {
    mpo_status st = check_live(h);
    if (st != MPO_OK) return st;
    if (!z) return fail(MPO_ERR_ARG, "z is NULL");
    return guarded(h, [&] { DISPATCH(h, E::observables(h, z, trace, nullptr)); });
}

mpo_status mpo_expect_z_all_noalloc(mpo_handle* h, double* z, double* trace) {
    mpo_status st = check_live(h);
    if (st != MPO_OK) return st;
    if (!z) return fail(MPO_ERR_ARG, "z is NULL");
    const size_t need = carve_obs_scratch(nullptr, h->n, h->chi_cap, nullptr);
    if (need > kStaticScratchBytes)
        return fail(MPO_ERR_ARENA, "n = %d, chi_cap = %d needs %zu bytes of scratch; the static scratch has %zu",
                    h->n, h->chi_cap, need, kStaticScratchBytes);
    char* base = (char*)static_scratch();
    if (!base) return MPO_ERR_HIP;
    ObsScratch w;
    carve_obs_scratch(base, h->n, h->chi_cap, &w);
    return guarded(h, [&] { DISPATCH(h, E::observables_in(h, w, z, trace, nullptr)); });
}

mpo_status mpo_bond_dims(mpo_handle* h, int* dims, int* center) {
    if (!h) return fail(MPO_ERR_ARG, "null handle");
    if (dims)
        for (int b = 0; b < h->n - 1; ++b) dims[b] = h->dims[b];
    if (center) *center = h->centre;
    return MPO_OK;
}

mpo_status run_brickwork(mpo_handle* h, int depth, const double* superops, int n_gates, int chi_max,
                         double cutoff, mpo_order order, int record_mask, double* S_out, double* Z_out,
                         double* trace_out, double* discarded_out) {
    mpo_status st = check_live(h);
    if (st != MPO_OK) return st;
    const int n = h->n;
    if (depth < 0) return fail(MPO_ERR_ARG, "depth must be >= 0");
    const long expect = (long)((depth + 1) / 2) * (n / 2) + (long)(depth / 2) * (n / 2 - 1);
    if (n_gates != expect)
        return fail(MPO_ERR_ARG, "n_gates = %d but a depth-%d brickwork on %d qubits has %ld", n_gates, depth, n, expect);
    if (n_gates > 0 && !superops) return fail(MPO_ERR_ARG, "superops is NULL");
    if (chi_max < 1 || chi_max > h->chi_cap) return fail(MPO_ERR_ARG, "chi_max %d out of [1, %d]", chi_max, h->chi_cap);
    if (!(cutoff >= 0.0) || !std::isfinite(cutoff)) return fail(MPO_ERR_ARG, "cutoff must be finite and >= 0");
    if (record_mask & ~3) return fail(MPO_ERR_ARG, "record_mask has unknown bits");
    if (order != MPO_ORDER_ASCENDING && order != MPO_ORDER_SNAKE)
        return fail(MPO_ERR_ARG, "unknown gate order %d", (int)order);
    if (!finite_all(superops, (size_t)n_gates * 512)) {
        h->poisoned = true;
        return fail(MPO_ERR_NUMERIC, "non-finite superoperator entry");
    }
    return guarded(h, [&] {
        DISPATCH(h, {
            using C = typename E::C;
            int g = 0, resident0 = 0, resident = 0;
            for (int t = 0; t < depth; ++t) {
                const int first = (t % 2 == 0) ? 0 : 1;
                const int last = first + 2 * ((n - 2 - first) / 2);
                const bool down = order == MPO_ORDER_SNAKE && (t % 2 == 1);
                for (int q = 0; q <= (last - first) / 2; ++q) {
                    const int s = down ? last - 2 * q : first + 2 * q;
                    if (g >= resident0 + resident) {
                        resident0 = g;
                        resident = std::min(kMaxSuper, n_gates - g);
                        HIPCHK(hipStreamSynchronize(h->st));
                        E::upload_super(h, superops + (size_t)g * 512, resident);
                    }
                    const C* Mg = (const C*)h->Mdev + (size_t)(g - resident0) * 256;
                    mpo_trunc_info inf = down ? E::apply_leftward(h, s, Mg, chi_max, cutoff)
                                              : E::apply(h, s, Mg, chi_max, cutoff);
                    if (discarded_out) discarded_out[g] = inf.discarded_weight;
                    ++g;
                }
                const bool rec_all = record_mask & 1;
                const bool rec_last = (record_mask & 2) && t == depth - 1;
                if (rec_all || rec_last) {
                    const int row = rec_all ? t : 0;
                    E::sweep_all(h, false);
                    if (S_out)
                        for (int b = 0; b < n - 1; ++b) S_out[(size_t)row * (n - 1) + b] = h->last_S[b];
                    double tr = 0.0;
                    E::observables(h, Z_out ? Z_out + (size_t)row * n : nullptr, &tr, nullptr);
                    if (trace_out) trace_out[row] = tr;
                }
            }
        });
    });
}

mpo_status mpo_set_tuning(mpo_handle* h, int block, int inner) {
    if (!h) return fail(MPO_ERR_ARG, "null handle");
    if ((block != 16 && block != 32) || inner < 1 || inner > 8)
        return fail(MPO_ERR_ARG, "block must be 16 or 32 and inner in [1, 8] (got %d, %d)", block, inner);
    h->jw.block = block;
    h->jw.inner = inner;
    return MPO_OK;
}

mpo_status mpo_set_default_tuning(mpo_precision prec, int chi_upto, int block, int inner) {
    if (prec != MPO_FP64 && prec != MPO_FP32_MFMA && prec != MPO_BF16X3)
        return fail(MPO_ERR_ARG, "unknown precision %d", (int)prec);
    if (chi_upto < 1 || (block != 16 && block != 32) || inner < 1 || inner > 8)
        return fail(MPO_ERR_ARG, "bad tuning entry (chi_upto %d, block %d, inner %d)", chi_upto, block, inner);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (TuneEntry& e : g_tune)
        if (e.prec == (int)prec && e.chi_upto == chi_upto) { e.block = block; e.inner = inner; return MPO_OK; }
    g_tune.push_back({(int)prec, chi_upto, block, inner});
    return MPO_OK;
}

mpo_status mpo_set_graphs(mpo_handle* h, int on) {
    if (!h) return fail(MPO_ERR_ARG, "null handle");
    if (on && !h->st) return fail(MPO_ERR_ARG, "captured sweeps need a non-null stream");
    h->jw.graphs = on != 0;
    return MPO_OK;
}

mpo_status mpo_set_precond(mpo_handle* h, int min_cols) {
    if (!h) return fail(MPO_ERR_ARG, "null handle");
    if (min_cols < 0) return fail(MPO_ERR_ARG, "min_cols must be >= 0 (0 = off), got %d", min_cols);
    if (min_cols > 0 && !h->jw.heev)
        return fail(MPO_ERR_ARG, "this handle has no eigen workspace (4 chi_cap < %d)", kHeevMinCols);
    h->jw.precond_min = min_cols;
    return MPO_OK;
}

mpo_status mpo_hermitian_eig(mpo_handle* h, int N, const double* G, double* w, double* V) {
    if (!h) return fail(MPO_ERR_ARG, "null handle");
    if (!G || !w || !V) return fail(MPO_ERR_ARG, "null argument");
    if (!h->jw.heev) return fail(MPO_ERR_ARG, "this handle has no eigen workspace (4 chi_cap < %d)", kHeevMinCols);
    if (N < 2 || N > h->hw.cap_n) return fail(MPO_ERR_ARG, "N = %d out of [2, %d]", N, h->hw.cap_n);
    if (!finite_all(G, (size_t)2 * N * N)) return fail(MPO_ERR_ARG, "non-finite matrix entry");
    return guarded(h, [&] {
        heev_host(N, G, w, V, h->hw, h->prof, h->st);
        for (int i = 0; i < N; ++i)
            if (!std::isfinite(w[i])) throw NumericError{"non-finite eigenvalue"};
    });
}

mpo_status mpo_run_brickwork_vidal(mpo_handle* h, int depth, const double* superops, int n_gates, int chi_max,
                                   double cutoff, double* S_out, double* discarded_out) {
    if (!h) return fail(MPO_ERR_ARG, "null handle");
    const int n = h->n;
    if (depth < 0) return fail(MPO_ERR_ARG, "depth must be >= 0");
    const long expect = (long)((depth + 1) / 2) * (n / 2) + (long)(depth / 2) * (n / 2 - 1);
    if (n_gates != expect)
        return fail(MPO_ERR_ARG, "n_gates = %d but a depth-%d brickwork on %d qubits has %ld", n_gates, depth, n, expect);
    if (n_gates > 0 && !superops) return fail(MPO_ERR_ARG, "superops is NULL");
    if (chi_max < 1 || chi_max > h->chi_cap) return fail(MPO_ERR_ARG, "chi_max %d out of [1, %d]", chi_max, h->chi_cap);
    if (!(cutoff >= 0.0) || !std::isfinite(cutoff)) return fail(MPO_ERR_ARG, "cutoff must be finite and >= 0");
    if (!finite_all(superops, (size_t)n_gates * 512)) return fail(MPO_ERR_ARG, "non-finite superoperator entry");
    mpo_status st = guarded(h, [&] {
        DISPATCH(h, E::run_vidal(h, depth, superops, n_gates, chi_max, cutoff, S_out, discarded_out));
    });
    if (st == MPO_OK) h->poisoned = false;
    return st;
}

mpo_status mpo_profile_enable(mpo_handle* h, int on) {
    if (!h) return fail(MPO_ERR_ARG, "null handle");
    h->prof.reset();
    h->prof.on = on != 0;
    h->jw.n_splits = h->jw.n_sweeps = h->jw.n_rounds = h->jw.n_rotations = h->jw.n_precond = h->jw.n_checks = 0;
    return MPO_OK;
}

mpo_status mpo_profile_read(mpo_handle* h, mpo_kernel_stat* out, int cap, int* count,
                            long long* svd_counters) {
    if (!h || !count) return fail(MPO_ERR_ARG, "null argument");
    if (cap > 0 && !out) return fail(MPO_ERR_ARG, "out is NULL");
    h->prof.collect();
    *count = K_COUNT;
    for (int k = 0; k < K_COUNT && k < cap; ++k) {
        std::snprintf(out[k].name, sizeof(out[k].name), "%s", kernel_name(k));
        out[k].launches = h->prof.launches[k];
        out[k].ms = h->prof.ms[k];
        out[k].flops = h->prof.flops[k];
        out[k].bytes = h->prof.bytes[k];
    }
    if (svd_counters) {
        svd_counters[0] = h->jw.n_splits;
        svd_counters[1] = h->jw.n_sweeps;
        svd_counters[2] = h->jw.n_rounds;
        svd_counters[3] = h->jw.n_rotations;
        svd_counters[4] = h->jw.n_precond;
        svd_counters[5] = h->jw.n_checks;
    }
    return MPO_OK;
}

mpo_status mpo_adjoint_workspace_bytes(int n, int depth, int chi_max, mpo_precision prec,
                                       int checkpoint_every, size_t* bytes) {
    if (!bytes) return fail(MPO_ERR_ARG, "bytes is NULL");
    size_t dummy = 0;
    mpo_status st = mpo_workspace_bytes(n, std::max(1, std::min(1024, 4 * chi_max)), prec, &dummy);
    if (st != MPO_OK) return st;
    if (depth < 1 || chi_max < 1 || chi_max > 1024) return fail(MPO_ERR_ARG, "depth >= 1 and 1 <= chi_max <= 1024 required");
    if (checkpoint_every < 0) return fail(MPO_ERR_ARG, "checkpoint_every must be >= 0 (0 = no recompute)");
    const int g = ((depth + 1) / 2) * (n / 2) + (depth / 2) * (n / 2 - 1);
    *bytes = adj_layout(n, depth, chi_max, prec, g, checkpoint_every).total;
    return MPO_OK;
}

mpo_status mpo_adjoint_brickwork(mpo_handle* h, int depth, const double* superops, int n_gates,
                                 int chi_max, double cutoff, int checkpoint_every, void* dev_work,
                                 size_t work_bytes, double* O_out, double* dO_dsuperop,
                                 int* costate_max_bond) {
    mpo_status st = check_live(h);
    if (st != MPO_OK) return st;
    const int n = h->n;
    if (depth < 1) return fail(MPO_ERR_ARG, "depth must be >= 1");
    const long expect = (long)((depth + 1) / 2) * (n / 2) + (long)(depth / 2) * (n / 2 - 1);
    if (n_gates != expect)
        return fail(MPO_ERR_ARG, "n_gates = %d but a depth-%d brickwork on %d qubits has %ld", n_gates, depth, n, expect);
    if (!superops || !O_out || !dO_dsuperop || !dev_work) return fail(MPO_ERR_ARG, "null argument");
    if (((uintptr_t)dev_work) & 255) return fail(MPO_ERR_ARG, "dev_work must be 256-byte aligned");
    if (chi_max < 1 || chi_max > h->chi_cap) return fail(MPO_ERR_ARG, "chi_max %d out of [1, %d]", chi_max, h->chi_cap);
    if (checkpoint_every < 0) return fail(MPO_ERR_ARG, "checkpoint_every must be >= 0 (0 = no recompute)");
    // tape slots, checkpoints and environments are sized by chi_max
    for (int b = 0; b < n - 1; ++b)
        if (h->dims[b] > chi_max)
            return fail(MPO_ERR_ARG, "bond %d of the current state has dimension %d > chi_max %d", b, h->dims[b], chi_max);
    if (!(cutoff >= 0.0) || !std::isfinite(cutoff)) return fail(MPO_ERR_ARG, "cutoff must be finite and >= 0");
    if (!finite_all(superops, (size_t)n_gates * 512)) return fail(MPO_ERR_ARG, "non-finite superoperator entry");
    const AdjLayout L = adj_layout(n, depth, chi_max, h->prec, n_gates, checkpoint_every);
    if (work_bytes < L.total) return fail(MPO_ERR_ARENA, "adjoint workspace has %zu bytes, %zu needed", work_bytes, L.total);
    return guarded(h, [&] {
        DISPATCH(h, Adjoint<typename E::C::value_type>::run(h, depth, superops, n_gates, chi_max, cutoff,
                                                           (char*)dev_work, L, O_out, dO_dsuperop,
                                                           costate_max_bond));
    });
}

mpo_status mpo_export(mpo_handle* h, void* host_buf, size_t cap, size_t* used) {
    if (!h || !used) return fail(MPO_ERR_ARG, "null argument");
    mpo_status st = MPO_OK;
    DISPATCH(h, { *used = E::export_size(h); });
    if (!host_buf) return MPO_OK;
    if (cap < *used) return fail(MPO_ERR_ARG, "buffer has %zu bytes, %zu needed", cap, *used);
    st = guarded(h, [&] { DISPATCH(h, E::do_export(h, (char*)host_buf)); });
    return st;
}

mpo_status mpo_import(mpo_handle* h, const void* host_buf, size_t len) {
    if (!h || !host_buf) return fail(MPO_ERR_ARG, "null argument");
    const int n = h->n;
    const size_t hdr_bytes = (size_t)(4 + n - 1) * 8;
    if (len < hdr_bytes) return fail(MPO_ERR_ARG, "snapshot too short");
    const int64_t* hdr = (const int64_t*)host_buf;
    if (hdr[0] != kMagicAny && hdr[0] != kMagicCanonical) return fail(MPO_ERR_ARG, "bad snapshot magic");
    if (hdr[3] < 0 || hdr[3] >= n) return fail(MPO_ERR_ARG, "snapshot centre out of range");
    if (hdr[1] != n) return fail(MPO_ERR_ARG, "snapshot has n = %lld, handle has %d", (long long)hdr[1], n);
    if (hdr[2] != h->basis) return fail(MPO_ERR_ARG, "snapshot basis differs from the handle's");
    size_t need = hdr_bytes;
    for (int b = 0; b < n - 1; ++b)
        if (hdr[4 + b] < 1 || hdr[4 + b] > h->chi_cap)
            return fail(MPO_ERR_ARG, "bond %d dimension %lld out of [1, %d]", b, (long long)hdr[4 + b], h->chi_cap);
    for (int s = 0; s < n; ++s) {
        const size_t cl = s == 0 ? 1 : hdr[4 + s - 1], cr = s == n - 1 ? 1 : hdr[4 + s];
        need += cl * 4 * cr * 16;
    }
    if (len < need) return fail(MPO_ERR_ARG, "snapshot has %zu bytes, %zu needed", len, need);
    if (!finite_all((const double*)((const char*)host_buf + hdr_bytes), (need - hdr_bytes) / 8))
        return fail(MPO_ERR_ARG, "snapshot holds non-finite values");
    mpo_status st = guarded(h, [&] { DISPATCH(h, E::do_import(h, (const char*)host_buf)); });
    if (st == MPO_OK) h->poisoned = false;
    return st;
}

}  // extern "C"

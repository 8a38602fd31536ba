/*
 * mpo.h - C ABI of libmpo, an MI355X (gfx950) engine for simulating noisy
 * one-dimensional random circuits with matrix product operators.
 *
 * Method: K. Noh, L. Jiang, B. Fefferman, "Efficient classical simulation of
 * noisy random quantum circuits in one dimension", Quantum 4, 318 (2020).
 * The density matrix is vectorised site by site (Sec. III.A: merged index
 * I = 2 i + i' for |i><i'|) and held as an MPS with physical dimension 4
 * (Eq. "MPO") in mixed canonical form.  A noisy two-qubit gate is one 16x16
 * superoperator M = N . U (Sec. III.B) applied to two neighbouring sites,
 * after which the bond is re-split by a truncated SVD (App. A; "Note added":
 * orthogonality centre moved locally, then a local truncation).
 *
 * Conventions for every entry point:
 *   - sites are 0-based, s in [0, n-1]; a gate acts on (s, s+1); bond b sits
 *     between sites b and b+1 (the paper's 1-based l is b+1);
 *   - host complex numbers are interleaved (re, im) float64, host matrices are
 *     row-major;
 *   - superoperator element [row][col] with row = 4*I_s + I_{s+1},
 *     col = 4*J_s + J_{s+1} (App. A, definition of M); in the Pauli basis the
 *     site index is P in {I,X,Y,Z} = {0,1,2,3} for the normalised operator
 *     sigma_P/sqrt(2);
 *   - the caller owns the device arena, the HIP stream and every host buffer;
 *     the library never allocates or frees device memory;
 *   - errors are returned as mpo_status with a message from mpo_last_error();
 *     an argument error leaves the state untouched; a numeric fault (non-finite
 *     values, SVD not converged) poisons the handle until mpo_init_product or
 *     mpo_import succeeds;
 *   - a handle is not thread-safe; distinct handles are independent.
 */
#ifndef MPO_H
#define MPO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpo_handle mpo_handle;

typedef enum {
    MPO_OK = 0,
    MPO_ERR_ARG = 1,      /* invalid argument; nothing changed               */
    MPO_ERR_ARENA = 2,    /* device arena too small                          */
    MPO_ERR_HIP = 3,      /* HIP runtime error                               */
    MPO_ERR_NUMERIC = 4,  /* NaN/Inf met; handle poisoned                    */
    MPO_ERR_NOCONV = 5,   /* SVD sweep limit reached; handle poisoned        */
    MPO_ERR_STATE = 6     /* handle poisoned by an earlier numeric fault     */
} mpo_status;

typedef enum {
    MPO_FP64 = 0,       /* complex128 tensors, FP64 MFMA contractions        */
    MPO_FP32_MFMA = 1,  /* complex64 tensors and contractions on FP32 MFMA;
                           the MFMA products are summed in FP32 over at most
                           32 terms and those partial sums in FP64;
                           truncation weights and entropy in FP64.  Singular
                           values with lambda^2 / sum lambda^2 <= 1e-11 are
                           at the mode's rounding floor and are never kept.
                           Any overall scale of the state is accepted: each
                           decomposition works on a power-of-two rescaled
                           copy of its matrix.                               */
    MPO_BF16X3 = 2      /* complex64 tensors; the two-site product, the
                           channel-fused theta, the centre moves and the
                           Jacobi Gram split each FP32 operand into BF16
                           hi + lo and sum three BF16 MFMA products in FP32
                           (about 16 significant bits, relative error of a
                           product up to about 3e-5).  Once the columns are
                           within 3e-3 of orthogonal the Jacobi Gram switches
                           to FP32 MFMA and the sweeps end at the FP32
                           tolerance, so isometries are as orthonormal as in
                           FP32 mode.  The Jacobi rotations, applied hundreds
                           of times to each column, stay on FP32 MFMA; the
                           eigen core, weights and entropy stay FP64.
                           Singular values with
                           lambda^2 / sum lambda^2 <= 1e-11 are at the mode's
                           rounding floor and are never kept.                 */
} mpo_precision;

typedef enum { MPO_BASIS_PAULI = 0, MPO_BASIS_COMPUTATIONAL = 1 } mpo_basis;

/* Result of one truncated split (App. A: keep the largest singular values).
 * kept: number of singular values kept, k = max(1, min(chi_max,
 *       #{alpha : lambda_alpha / ||lambda||_2 > cutoff})), norm over the full
 *       pre-truncation spectrum;
 * discarded_weight: sum of lambda^2 over the dropped values;
 * total_weight: sum of lambda^2 over all values (= ||theta'||_F^2);
 * entropy: MPO entanglement entropy of the kept values (Sec. III.C, Eq. S_l),
 *          -sum w log2 w with w = lambda^2 / sum_kept lambda^2.            */
typedef struct {
    int kept;
    double discarded_weight;
    double total_weight;
    double entropy;
} mpo_trunc_info;

/* Device bytes needed for a chain of n sites with bond cap chi_cap.  The arena
 * holds n+2 site slots of 4*chi_cap^2 complex values plus the SVD workspace. */
mpo_status mpo_workspace_bytes(int n, int chi_cap, mpo_precision prec, size_t *bytes);

/* Create a handle over a caller-owned device arena (256-byte aligned, at
 * least mpo_workspace_bytes) and HIP stream (NULL = default stream).
 * n even and >= 2 (Sec. II.A), 1 <= chi_cap <= 1024.  The state starts as
 * |0..0><0..0| (Sec. IV.A initial MPO).                                      */
mpo_status mpo_create(int n, int chi_cap, mpo_precision prec, mpo_basis basis,
                      void *dev_arena, size_t arena_bytes, void *hip_stream,
                      mpo_handle **out);
void mpo_destroy(mpo_handle *h);

/* Product state |x><x| with x given as n bytes in {0,1}; NULL = all zero
 * (Sec. IV.A: lambda = (1,0,...), Gamma = 1 at alpha = I = 0).  All bond
 * dimensions become 1, the orthogonality centre is site 0.                   */
mpo_status mpo_init_product(mpo_handle *h, const unsigned char *bits);

/* Apply a 16x16 complex superoperator (host, row-major, interleaved, in the
 * handle's basis) to sites (site, site+1): move the orthogonality centre to
 * `site` (exact), contract the two sites, apply the map, split by a truncated
 * SVD (App. A truncation; "Note added" local update).  Afterwards site is a
 * left isometry and site+1 the centre.  The host sequences the SVD: it reads
 * the convergence measure of every Jacobi sweep and the kept count of every
 * split back from the device, so the call synchronises the handle's stream a
 * few times per split whether info is NULL or not (the call is not capturable
 * in a HIP graph).  info != NULL receives the split's result.               */
mpo_status mpo_apply_2q_channel(mpo_handle *h, int site, const double *superop,
                                int chi_max, double cutoff, mpo_trunc_info *info);

/* Move the orthogonality centre to `center` by exact re-gauging (no
 * truncation beyond singular values below the working precision).            */
mpo_status mpo_canonicalize(mpo_handle *h, int center);

/* MPO entanglement entropy S_b (Sec. III.C, Eq. S_l, log base 2) from the
 * Schmidt values of the current state at bond b in [0, n-2]; bond = -1 writes
 * all n-1 values (one canonical sweep).  Synchronises.                       */
mpo_status mpo_bond_entropy(mpo_handle *h, int bond, double *S);

/* Schmidt values lambda^[b+1] of the vectorised state at bond b (Sec. III.A:
 * the MPO written in Vidal's form, lambda as Schmidt coefficients; the same
 * values give S_b of Sec. III.C), descending, from a fresh exact re-gauge of
 * the current state; at most cap of them are written, *count = number
 * available.  Errors: MPO_ERR_ARG for a bond outside [0, n-2], a NULL count,
 * or cap > 0 with lam NULL.  Synchronises.                                   */
mpo_status mpo_singular_values(mpo_handle *h, int bond, double *lam, int cap, int *count);

/* Tr[P rho] / Tr[rho] for a Pauli string (n codes 0=I 1=X 2=Y 3=Z) by
 * transfer contraction (Sec. III.D); im is a Hermiticity diagnostic.        */
mpo_status mpo_expect_pauli(mpo_handle *h, const unsigned char *pauli, double *re, double *im);

/* Total probability Tr[rho] (Sec. III.D); below 1 after truncation.          */
mpo_status mpo_trace(mpo_handle *h, double *re, double *im);

/* All <Z_i> = Tr[Z_i rho]/Tr[rho] (n values) and Tr[rho].                    */
mpo_status mpo_expect_z_all(mpo_handle *h, double *z, double *trace);

/* mpo_expect_z_all for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same transfer contraction, with its FP64 environments in a static
 * device array of the library (8 MiB per GPU, held until the process ends)
 * instead of the handle's arena.  The call allocates nothing and performs no
 * allocating library call; the array's device address is looked up on the
 * first call on each device.  Needs 2 (n+1) chi_cap + 65 chi_cap + 5 (n+2)
 * complex FP64 values of scratch (each part 256-byte aligned), at most 8 MiB:
 * a larger handle is MPO_ERR_ARENA before any launch.  Every call on a GPU
 * shares that GPU's array and leaves its contents behind (every value the
 * contraction reads is written first in the same call): calls that overlap on
 * one GPU, from several threads or streams, race and must not be issued.
 * The current device must be the handle's.  Synchronises.                   */
mpo_status mpo_expect_z_all_noalloc(mpo_handle *h, double *z, double *trace);

/* Output probability of a computational-basis measurement (Sec. III.D):
 * P(x) = Tr[|x><x| rho], a contraction of the MPO with one projector vector
 * per site.  bits: n values in {0,1}, bits[0] is the leftmost qubit.  The value
 * is that of the held (possibly truncated) state, not divided by Tr rho; im is
 * a rounding diagnostic.  Summed over all x it gives Tr rho (Sec. III.D).
 * Errors: MPO_ERR_ARG for a null pointer or a bit outside {0,1}.             */
mpo_status mpo_probability(mpo_handle *h, const unsigned char *bits, double *re, double *im);

/* Bit strings drawn by sequential conditional sampling (Sec. III.D, sampling
 * via marginals): the marginal of x_1 with every later site summed out, then
 * the conditional of each next bit given the drawn prefix.  The caller supplies
 * the randomness: uniforms is n_samples x n values in [0, 1), sample-major
 * (uniforms[s*n + k] draws bit k of sample s); bit k is 0 when
 * uniforms[s*n+k] < P(0 | prefix) / (P(0 | prefix) + P(1 | prefix)), else 1.
 * A truncated rho need not be positive: a negative marginal is taken as 0 and
 * the sample is counted in *clamped; if both marginals vanish the bit is 0.
 * Outputs (host): bits (n_samples x n, sample-major), prob (n_samples values of
 * P(x) of each drawn string, unnormalised as in mpo_probability; may be NULL),
 * clamped (may be NULL).  The samples are processed in chunks sized to the
 * handle's scratch (theta buffers; the state itself is not modified).
 * Errors: MPO_ERR_ARG for n_samples < 1, null inputs or a uniform outside
 * [0, 1); MPO_ERR_ARENA if the scratch cannot hold even one sample.          */
mpo_status mpo_sample(mpo_handle *h, int n_samples, const double *uniforms, unsigned char *bits,
                      double *prob, int *clamped);

/* Current bond dimensions chi_b (n-1 values; the range of the alpha_b index
 * of Sec. III.A, dynamic here instead of a fixed padded chi) and the site of
 * the orthogonality centre of the mixed canonical form ("Note added").  dims
 * and center may be NULL.  Host bookkeeping only: no GPU work.              */
mpo_status mpo_bond_dims(mpo_handle *h, int *dims, int *center);

/* Order of the gates within a time step.  Gates of one step act on disjoint
 * pairs, so without truncation every order gives the same state (Sec. II.A);
 * under truncation the order is part of the algorithm.  ASCENDING applies them
 * from the left (the reading of Sec. IV.A's sequential application).  SNAKE
 * applies odd time steps ascending and even ones descending, splitting each
 * descending gate with the centre left on its left site, so the centre never
 * travels back across the chain between steps.                             */
typedef enum { MPO_ORDER_ASCENDING = 0, MPO_ORDER_SNAKE = 1 } mpo_order;

/* Brickwork evolution (Sec. II.A, Sec. IV.A): time step t = 1..depth puts a
 * gate on (0,1),(2,3),... for odd t and on (1,2),(3,4),... for even t, in the
 * given order.  superops: n_gates x 16 x 16 complex in schedule order (time
 * step by time step; within a descending step from the rightmost gate to the
 * leftmost), n_gates = ceil(D/2) n/2 + floor(D/2) (n/2-1), else MPO_ERR_ARG.
 * record_mask bit 0: after every time step write S_b for all n-1 bonds to
 * S_out[t*(n-1)+b], <Z_i> to Z_out[t*n+i] and Tr rho to trace_out[t];
 * bit 1: the same only after the last time step (index 0).  Outputs may be
 * NULL when not recorded.  discarded_out (n_gates values or NULL) receives
 * the discarded weight of every gate.  Evolution continues from the current
 * state.  An unknown order or record bit is MPO_ERR_ARG.  Synchronises.     */
mpo_status run_brickwork(mpo_handle *h, int depth, const double *superops, int n_gates,
                         int chi_max, double cutoff, mpo_order order, int record_mask,
                         double *S_out, double *Z_out, double *trace_out,
                         double *discarded_out);

/* The paper's own update (App. A) for comparison with the local one: the
 * state held in the Gamma-lambda form (Sec. III.A, lambda the Schmidt values
 * of every bond), each noisy gate applied to B = lambda Gamma lambda Gamma
 * lambda and split by the truncated SVD, then the canonical form of the whole
 * chain restored by SVD sweeps to the left (B_<-) and to the right (B_->),
 * with every Gamma recovered by dividing by the new lambda (Gamma <- W /
 * lambda').  Singular values at or below 1e-14 of the largest are removed
 * before any division.  n - 1 decompositions per gate, O(n chi^3) per gate
 * against the O(chi^3) of mpo_apply_2q_channel (the "Note added"); in exact
 * arithmetic the two truncate the same Schmidt values.  Starts from
 * |0..0><0..0| (the current state is replaced), applies the ascending
 * brickwork of run_brickwork (same superops layout and n_gates rule), writes
 * S_b of every bond after every time step to S_out[t*(n-1)+b] (read from the
 * lambdas, no extra sweep) and the discarded weight of every gate to
 * discarded_out (either may be NULL), and leaves the handle in the mixed
 * canonical form with the centre at n-1.  Errors as run_brickwork.
 * Synchronises.                                                             */
mpo_status mpo_run_brickwork_vidal(mpo_handle *h, int depth, const double *superops, int n_gates,
                                   int chi_max, double cutoff, double *S_out, double *discarded_out);

/* Host snapshot of the state.  Format: int64 header {magic, n, basis, center,
 * chi_0 .. chi_{n-2}} then per site the (chi_l, 4, chi_r) tensor, row-major,
 * complex128.  Exports carry magic 0x4d504f32 ("MPO2": sites left of center
 * are left isometries, sites right of it right isometries).  host_buf may be
 * NULL to query *used.                                                       */
mpo_status mpo_export(mpo_handle *h, void *host_buf, size_t cap, size_t *used);
/* Load a snapshot.  Magic 0x4d504f31 ("MPO1"): tensors in any gauge, brought
 * into canonical form by exact moves.  Magic 0x4d504f32: trusted to be in
 * mixed canonical form about the stored center, loaded as is.               */
mpo_status mpo_import(mpo_handle *h, const void *host_buf, size_t len);

/* Noisy Haar gate superoperator, host only: U = Haar unitary from one complex
 * Ginibre draw (re, im: 4x4 row-major float64; Q of a QR with positive R
 * diagonal, Mezzadri 2007), M = N2[p] . U in the given basis (Sec. II.B
 * depolarizing channel, Sec. III.B M = N . U, App. A element definition).
 * out: 16x16 complex interleaved row-major.  Also writes U (4x4 complex
 * interleaved) to u_out unless NULL.                                         */
mpo_status mpo_build_superop(const double *re, const double *im, double p, mpo_basis basis,
                             double *out, double *u_out);

/* Batched evolution of independent circuits (the paper averages over N_s
 * independent random circuits, Sec. IV.A).  Each circuit is an ascending
 * brickwork as in run_brickwork, starting from |0..0><0..0|.
 *   use_graph: 1 = Jacobi sweeps replayed from captured HIP graphs
 *     (mpo_set_graphs) on every circuit's handle; streams must be non-null.
 *   superops_concat: all circuits' superoperators (16x16 complex each),
 *     circuit c using gates [gate_offset, gate_offset + n_gates(n, depth)).
 *   record_mask: 0 or 2 = observables after the last time step only, 1 = after
 *     every time step (R = depth rows; R = 1 for depth 0 or the last step).
 *   results: per circuit at result_offset, mpo_batch_result_doubles(n, depth,
 *     record_mask) = 2 n R + 2 values: S_b (R rows of n-1), <Z_i> (R rows of
 *     n), Tr rho (R), then the summed discarded weight and the largest bond
 *     dimension reached (as a double).
 * Work is spread over n_streams caller-owned HIP streams (n_streams >= 1),
 * one host worker thread per stream; circuits are taken largest first
 * (n * depth * chi_max^3).  The arena is split into n_streams equal slices,
 * each of mpo_batch_workspace_bytes(...) / n_streams bytes.  A circuit's
 * computation does not depend on which stream runs it, so the results equal
 * those of separate run_brickwork calls.  Synchronises all streams.          */
typedef struct {
    int n, depth, chi_max;
    double cutoff;
    size_t gate_offset;     /* first superoperator of this circuit            */
    size_t result_offset;   /* first double of this circuit in results        */
} mpo_batch_desc;
mpo_status mpo_batch_workspace_bytes(const mpo_batch_desc *circuits, int count,
                                     mpo_precision prec, int n_streams, size_t *bytes);
int mpo_batch_result_doubles(int n, int depth, int record_mask);
mpo_status mpo_batch_run(const mpo_batch_desc *circuits, int count,
                         const double *superops_concat, size_t n_superops,
                         mpo_precision prec, mpo_basis basis,
                         void *dev_arena, size_t arena_bytes,
                         void *const *hip_streams, int n_streams, int use_graph,
                         int record_mask, double *results);

/* Gradient of O = sum_i Tr[Z_i rho_D] (unnormalised, so linear in rho) with
 * respect to every gate superoperator, with the truncation projectors frozen.
 * Truncation at gate g keeps the top-k left Schmidt vectors at its bond (App. A);
 * frozen at the forward point it is the orthogonal projector
 * P_g = (Phi_g Phi_g^H) (x) 1 onto the kept left vectors, and exact re-gauging
 * moves are identities, so rho_D = P_G M_G ... P_1 M_1 rho_0 is linear in each
 * M_g.  Runs the brickwork of run_brickwork (same superops, chi_max, cutoff)
 * from the handle's current state, recording per time step the state at its
 * start, every pre-gate centre tensor and the left isometries after its last
 * gate; then propagates the co-state mu_G = w, lambda_g = P_g mu_g,
 * mu_{g-1} = M_g^H lambda_g backwards as an MPS (bond <= min(1024, 4 chi_max);
 * the largest bond reached is written to *costate_max_bond unless NULL).
 *   O_out: O at the forward point;
 *   dO_dsuperop: n_gates x 16 x 16 complex, dO/dM_g[row][col] such that
 *     O = sum_{row,col} M_g[row][col] * dO_dsuperop_g[row][col] for every g;
 *   dev_work: caller device memory, 256-byte aligned, of at least
 *     mpo_adjoint_workspace_bytes(n, depth, chi_max, prec) bytes.
 * The handle ends in the forward's final state.  Synchronises.               */
mpo_status mpo_adjoint_workspace_bytes(int n, int depth, int chi_max, mpo_precision prec,
                                       int checkpoint_every, size_t *bytes);
mpo_status mpo_adjoint_brickwork(mpo_handle *h, int depth, const double *superops, int n_gates,
                                 int chi_max, double cutoff, int checkpoint_every,
                                 void *dev_work, size_t work_bytes,
                                 double *O_out, double *dO_dsuperop, int *costate_max_bond);

/* Launch mode of the Jacobi sweeps of a handle.  on = 1: each sweep (norm
 * sort, every round's pair Gram / eigen-solver / update launches, and the
 * convergence test, which runs on the device) is captured once per matrix
 * shape into a HIP graph and replayed; several sweeps are queued between two
 * reads of the convergence flag, and the launches of a sweep queued after
 * convergence return at once.  Results are bit-identical to on = 0 (direct
 * launches, one read per sweep).  Needs the handle's stream to be non-null
 * (MPO_ERR_ARG otherwise).  Per-kernel profiling uses direct launches.      */
mpo_status mpo_set_graphs(mpo_handle *h, int on);

/* Tunables of the blocked one-sided Jacobi: block width (16 or 32 columns, a
 * block pair is twice that) and inner FP64 sweeps per block pair (1..8).
 * mpo_set_tuning sets them on one handle; mpo_set_default_tuning records an
 * entry used by every later mpo_create of that precision whose chi_cap is at
 * most chi_upto (the smallest such chi_upto wins; environment overrides
 * MPO_JACOBI_BLOCK / MPO_JACOBI_INNER still apply after it).  Entries come
 * from the autotuner (paper_2003_13163_amd/autotune.py), which times the
 * candidates on in-situ gates.  Errors: MPO_ERR_ARG for other values.       */
mpo_status mpo_set_tuning(mpo_handle *h, int block, int inner);
mpo_status mpo_set_default_tuning(mpo_precision prec, int chi_upto, int block, int inner);

/* Starting basis of the truncated split (App. A: SVD of the two-site block).
 * A split of an m x N block with N >= min_cols first computes the Gram matrix
 * G = theta'^H theta' (FP64), its eigenvectors V (Householder
 * tridiagonalisation, divide and conquer on the tridiagonal), and hands
 * theta' V, whose columns are orthogonal to about the FP64 eigen-solver's
 * accuracy relative to their own norms, to the one-sided Jacobi.  In FP64
 * storage all N columns are formed and the sweeps polish them (they still
 * decide convergence, the values and the isometries); in FP32 storage only
 * the columns of the chi_max + 64 largest eigenvalues are formed, one FP64
 * Gram of them certifies their orthogonality to the sweeps' tolerance (the
 * sweeps run only if it does not), and the weight of the other columns (the
 * sum of their eigenvalues) enters the truncation as discarded weight.  Every
 * mode computes this start in FP64.  min_cols = 0 turns it off.  Default 1024 (environment override MPO_PRECOND_MIN).  Handles with
 * 4 chi_cap < 512 have no eigen workspace: min_cols > 0 is MPO_ERR_ARG there. */
mpo_status mpo_set_precond(mpo_handle *h, int min_cols);

/* The eigen-solver of mpo_set_precond on a host matrix, for tests: G is an
 * N x N Hermitian matrix (row-major, interleaved complex, caller-owned), w
 * receives the N eigenvalues in ascending order and V (row-major, interleaved
 * complex, N x N) the eigenvectors as columns.  2 <= N <= 4 chi_cap; uses the
 * handle's arena and stream (synchronises).  MPO_ERR_ARG: no eigen
 * workspace, N out of range, non-finite input.  The state is unchanged.     */
mpo_status mpo_hermitian_eig(mpo_handle *h, int N, const double *G, double *w, double *V);

/* Instrumentation: per-kernel-class timing with HIP events recorded on the
 * handle's stream around every launch, plus the algorithmic flop and byte
 * counts of those launches (real flops; complex MAC = 8).  Enabling resets
 * the counters.  Timing adds two event records per launch.                   */
typedef struct {
    char name[24];      /* theta_channel, jacobi_gram, jacobi_eig64, ...      */
    long long launches;
    double ms;          /* summed event-measured duration                    */
    double flops;       /* algorithmic real flops of those launches          */
    double bytes;       /* algorithmic HBM bytes of those launches           */
} mpo_kernel_stat;
mpo_status mpo_profile_enable(mpo_handle *h, int on);
/* Synchronises.  Writes up to cap entries; *count = number of kernel classes.
 * svd_counters (6 values or NULL): splits, Jacobi sweeps, Jacobi rounds,
 * rotated block pairs, splits started from the Gram eigenvectors, and of
 * those the splits their Gram certificate finished without a sweep.         */
mpo_status mpo_profile_read(mpo_handle *h, mpo_kernel_stat *out, int cap, int *count,
                            long long *svd_counters);

/* Last error message of the calling thread ("" if none).                     */
const char *mpo_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MPO_H */

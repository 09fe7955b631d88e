/*
 * casci.h -- C ABI of the MI355X (gfx950) string-based CASCI library.
 *
 * What it computes. The lowest eigenpairs of the fermionic Hamiltonian of
 * eq. (hamiltonian) (Sec. II of Evangelista et al., "Forte: a suite of
 * advanced multireference quantum chemistry methods")
 *
 *     H = V + sum_pq h_pq a+_p a_q + 1/4 sum_pqrs <pq||rs> a+_p a+_q a_s a_r
 *
 * restricted to the complete active space of norb spatial orbitals holding
 * nalpha alpha and nbeta beta electrons (Sec. II.A.1). Determinants are
 * products of an alpha string and a beta string, |Ia> (x) |Ib>, and a CI
 * vector is the matrix C[Ia][Ib] (Sec. II.A.1, string-based CI). The
 * library computes sigma = H C (the sigma build of Sec. II.A.1) and runs a
 * Davidson-Liu eigensolver on top of it (Sec. II.A.1).
 *
 * Conventions fixed by this header (the paper leaves them open):
 *  - A string is a 64-bit mask, bit p = orbital p occupied (Sec. III.C).
 *  - Strings of one spin are numbered 0..N-1 in ascending integer order of
 *    their masks (a gap-free address, Sec. II.A.1); string 0 is the aufbau
 *    string 0..n-1.
 *  - Determinant (Ia, Ib) = a+_{Ia...} a+_{Ib...} |->: all alpha creators to
 *    the left of all beta creators, each group in ascending orbital order
 *    (the canonical operator order of Sec. III.C). This fixes the sign of
 *    every CI coefficient. Its address is Ia*Nb + Ib (C is row-major).
 *  - Two-electron integrals are passed in chemists' notation (pq|rs), which
 *    is the paper's <pr|qs> (Sec. III.B), stored at ((p*n+q)*n+r)*n+s.
 *
 * Memory. Every pointer argument is accompanied by a `mem` flag: HOST
 * pointers are copied in/out by the library (the call then synchronises the
 * context stream), DEVICE pointers must live on the context's device and
 * are used in place, ordered on the context stream. Inputs are borrowed for
 * the duration of the call only; the library keeps its own copies.
 *
 * Errors. Every call returns a status code (CASCI_OK = 0, warnings > 0,
 * errors < 0) and never aborts or prints. The message of the last error of
 * a context is available from casci_last_error. A failed call leaves the
 * context in its previous valid state unless stated otherwise.
 *
 * Threads. A context must not be used from two threads at once; distinct
 * contexts are independent.
 */
#ifndef CASCI_H
#define CASCI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define CASCI_OK 0
#define CASCI_NOCONV 1          /* davidson: max_iter reached; results are filled */
#define CASCI_E_ARG (-1)        /* invalid argument (sizes, symmetry, null pointer) */
#define CASCI_E_STATE (-2)      /* call order: integrals / strings missing or mismatched */
#define CASCI_E_NOMEM (-3)      /* predicted or actual device allocation failure */
#define CASCI_E_DEVICE (-4)     /* HIP runtime error; message in casci_last_error */
#define CASCI_E_NONFINITE (-5)  /* NaN or Inf in the input */
#define CASCI_E_UNSUPPORTED (-6)

/* where a pointer lives */
#define CASCI_MEM_HOST 0
#define CASCI_MEM_DEVICE 1

/* element types of CI vectors / arithmetic of the alpha-beta contraction */
#define CASCI_F64 0
#define CASCI_F32 1
#define CASCI_BF16 2

/* Davidson preconditioners */
#define CASCI_PRECOND_DIAG 0    /* t = -r / (H_II - theta) */
#define CASCI_PRECOND_OLSEN 1   /* diagonal + Olsen's correction along x */
#define CASCI_PRECOND_MLP 2     /* learned correction, Olsen fallback */

/* spin targets */
#define CASCI_SPIN_ANY 0        /* lowest roots of the whole (nalpha, nbeta) space */
#define CASCI_SPIN_SINGLET 1    /* S = 0 roots (needs nalpha == nbeta) */

#define CASCI_MAX_ROOTS 32

typedef struct casci_ctx casci_ctx;

/*
 * Create a context on HIP device `device` (>= 0), ordering all work on
 * `hip_stream` (a hipStream_t; NULL = a stream owned by the context).
 * device = -1 gives a validate-only context: every call checks its
 * arguments and state exactly as on a GPU and then returns
 * CASCI_E_UNSUPPORTED instead of launching work (no HIP call is made).
 * Returns CASCI_E_ARG for out == NULL, CASCI_E_DEVICE if the device cannot
 * be used. On error *out is NULL.
 */
int casci_create(casci_ctx** out, int device, void* hip_stream);

/*
 * Device memory cache: blocks of 64 MiB and more that the library frees
 * (the Davidson basis, vector-sized work buffers) are kept for later
 * requests of about the same size instead of being returned to the driver,
 * at most three quarters of a device's memory (the least recently released
 * blocks go first); an allocation that fails empties the cache of its device
 * and is retried. casci_release_cache returns the cached
 * blocks of `device` (-1: every device) to the driver, casci_cached_bytes
 * reports how many bytes are held. Not for use while another thread is in a
 * library call on that device.
 */
int casci_release_cache(int device);
int64_t casci_cached_bytes(int device);

/* Free every buffer of the context (NULL is a no-op). */
void casci_destroy(casci_ctx* ctx);

/* Message of the last error on this context ("" if none); owned by ctx. */
const char* casci_last_error(const casci_ctx* ctx);

/*
 * set_integrals: h (norb x norb, row-major, symmetric), eri (norb^4,
 * chemists' (pq|rs)), e_core = the scalar V of eq. (hamiltonian). mem =
 * CASCI_MEM_HOST or CASCI_MEM_DEVICE for h and eri. The arrays are copied.
 * eri needs the symmetry of a Hermitian Hamiltonian, (pq|rs) = (qp|sr) =
 * (rs|pq); the 8-fold symmetry of real-orbital integrals ((pq|rs) = (qp|rs)
 * as well) is detected and lets the alpha-beta term fold its pair rows.
 * Without it -- dressed integrals, such as the similarity-transformed
 * Hamiltonian whose model-space diagonalisation is the reference relaxation
 * of Sec. II.C -- the alpha-beta term runs over all ordered orbital pairs
 * (the same sigma and Davidson otherwise). Checks: 1 <= norb <= 64,
 * finiteness (CASCI_E_NONFINITE), symmetry of h and the 4-fold symmetry of
 * eri to 1e-12 * max|value| (CASCI_E_ARG). If strings for a different norb
 * exist the call fails with CASCI_E_STATE. Invalidates all
 * integral-dependent device data (same-spin operators, diagonal,
 * pair-integral matrices).
 */
int casci_set_integrals(casci_ctx* ctx, int norb, const double* h, const double* eri,
                        double e_core, int mem);

/*
 * build_strings: enumerate the nalpha- and nbeta-electron strings of norb
 * orbitals and their single-substitution lists (Sec. II.A.1: gap-free
 * string addresses and precomputed substitution lists), on the device.
 * Requires 0 <= nalpha, nbeta <= norb <= 64 and fewer than 2^31 strings
 * per spin; if integrals are set, norb must match (CASCI_E_STATE). The
 * device memory that sigma/davidson will need for one vector pair is
 * predicted first; CASCI_E_NOMEM leaves no partial state.
 */
int casci_build_strings(casci_ctx* ctx, int nalpha, int nbeta, int norb);

/*
 * dims[0..7] = {Na, Nb, Ndet, sa, sb, ra, rb, norb}: string counts,
 * determinant count, single-substitution list length per string
 * (s = n_e (norb - n_e + 1), diagonal E_pp included) and nonzeros per row
 * of the same-spin operator (r = 1 + n_e(n-n_e) + C(n_e,2) C(n-n_e,2)).
 */
int casci_get_dims(const casci_ctx* ctx, int64_t* dims);

/* Copy the strings of one spin (0 = alpha, 1 = beta) to host out[N]. */
int casci_get_strings(casci_ctx* ctx, int spin, uint64_t* out);

/*
 * Copy the single-substitution list of one spin to host arrays of N*s
 * entries: for string I, entry e = I*s + k holds (p, q, J, sign) with
 * <I| a+_p a_q |J> = sign != 0; p runs over the occupied orbitals of I in
 * ascending order and, for each p, q over {unoccupied orbitals of I} U {p}
 * ascending. Any output pointer may be NULL.
 */
int casci_get_single_list(casci_ctx* ctx, int spin, int32_t* J, int8_t* sign, uint8_t* p,
                          uint8_t* q);

/*
 * Copy the same-spin operator of one spin to host arrays of N*r entries:
 * F(I,J) = sum_pq k_pq <I|E_pq|J> + 1/2 sum_pqrs (pq|rs) <I|E_pq E_rs|J>
 * with k_pq = h_pq - 1/2 sum_r (pr|rq), E restricted to that spin; this is
 * H of eq. (hamiltonian) for the (n_e, 0) system without V. Row I lists its
 * r nonzero columns in ascending order (col) with their values (val).
 * Requires integrals and strings.
 */
int casci_get_same_spin_operator(casci_ctx* ctx, int spin, int32_t* col, double* val);

/* Diagonal H_II (V included) of every determinant -> out[Ndet] (host or device). */
int casci_get_diagonal(casci_ctx* ctx, double* out, int mem);

/*
 * Addresses (row-major into [Na][Nb]) of the `want` lowest diagonal elements
 * H_II (eq. (hamiltonian)), ascending by value, ties by lower address: the
 * determinants the Davidson start space is built from. out: host int64
 * [want]; 0 <= want <= number of determinants, else CASCI_E_ARG.
 */
int casci_lowest_diagonal(casci_ctx* ctx, int64_t want, int64_t* out);

/*
 * sigma: sigma = H C for one CI vector (the sigma build of Sec. II.A.1).
 * C and sigma are Na x Nb row-major arrays of `dtype` (CASCI_F64, or
 * CASCI_F32 for single-precision storage). ab_prec selects the arithmetic
 * of the alpha-beta contraction: CASCI_F64 (FP64 MFMA), CASCI_F32 (FP32
 * MFMA) or CASCI_BF16 (BF16 MFMA, FP32 accumulate); the alpha-alpha /
 * beta-beta terms accumulate in FP64 (in FP32 in the row-blocked gather of a
 * BF16 build, see casci_get_tuning). FP32 storage on the device with
 * ab_prec F32/BF16 keeps every vector-sized buffer in FP32 (no FP64 copy:
 * the large-active-space path); other FP32 cases convert to FP64 inside.
 * sigma is overwritten, never accumulated. C and sigma must not overlap.
 */
int casci_sigma(casci_ctx* ctx, const void* C, void* sigma, int dtype, int ab_prec, int mem);

/*
 * sigma = H C for a CI vector of definite transposition parity, C = parity C^T
 * (parity = +1 or -1; needs nalpha = nbeta and FP64 storage). For equal
 * electron counts, transposing C (swapping the alpha and beta strings of every
 * determinant) commutes with H, and with the determinant phase of this header
 * it maps a spin-S state to (-1)^S times itself: singlets have parity +1,
 * triplets -1. The beta-beta term is then parity times the transpose of the
 * alpha-alpha term, so one same-spin gather serves both spins; the Davidson
 * solver builds every sigma this way when nalpha = nbeta. ab_prec as in
 * casci_sigma (F32/BF16: the same-spin gather reads an FP32 copy of C and
 * accumulates in FP64). The parity of C is the caller's promise and is not
 * checked: for a C without it the result is F_a C + parity (F_a C)^T + the
 * alpha-beta term, not H C.
 */
int casci_sigma_parity(casci_ctx* ctx, const double* C, double* sigma, int ab_prec, int parity, int mem);

/*
 * Allocation-free sigma, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): sigma = H C as casci_sigma / casci_sigma_parity compute it
 * (parity 0: any C; parity +1 / -1: C = parity C^T, nalpha = nbeta), for FP64
 * device vectors C and sigma (Na x Nb, row-major, on the context's device),
 * ordered on the context stream. Its work buffers (the transposes, the
 * alpha-beta term, the row maxima and the low-precision copies of C) live in
 * a 64 MiB static device array that the library holds on every GPU it runs on
 * until the process ends; the call makes no allocation of any kind. Limits
 * and preconditions:
 *  - the string space must fit the scratch: 24 Ndet + 8 Na bytes (FP64,
 *    parity 0), 8 Ndet + 8 Na (FP64, parity +-1), about 30 Ndet (F32/BF16,
 *    parity 0); CAS(12,12) fits, CAS(14,14) does not -> CASCI_E_UNSUPPORTED;
 *  - the operators and tables must already exist: run casci_sigma once with
 *    the same ab_prec after set_integrals / build_strings (CASCI_E_STATE
 *    otherwise);
 *  - every call on a GPU shares that GPU's scratch, which keeps the last
 *    call's contents: calls that overlap in time on one GPU (two streams, two
 *    threads) race and give wrong results; calls ordered on one stream are safe.
 */
int casci_sigma_noalloc(casci_ctx* ctx, const double* C, double* sigma, int ab_prec, int parity);

/*
 * Reduced density matrices of a real CI vector C (Na x Nb FP64, host or
 * device per mem; it need not be normalised: the matrices scale with |C|^2),
 * the quantities the orbital optimisation and perturbation theories built on
 * the CASCI solve consume (Sec. II.A.1; Sec. II.B uses the one- and
 * two-particle density matrices of the CI vectors). Spin-resolved, host outputs:
 *   g1[s][p][q]        = <C| a+_{p s} a_{q s} |C>,  s = 0 alpha, 1 beta      (2 n^2)
 *   g2[k][p][q][r][u]  = <C| a+_{p s} a+_{r t} a_{u t} a_{q s} |C>          (3 n^4)
 *                        k = 0: (s,t) = (alpha,alpha), 1: (alpha,beta), 2: (beta,beta)
 * g2 = NULL skips the two-particle matrix. With real orbitals the energy is
 * E = V + sum_pq h_pq gamma_pq + 1/2 sum_pqru (pq|ru) Gamma_pqru with the
 * spin sums of casci_rdm_spin_free. Needs strings (not integrals). Works on
 * blocks of alpha strings holding at most 512 MiB of pair-excitation rows.
 */
int casci_rdm(casci_ctx* ctx, const double* C, int mem, double* g1, double* g2);

/*
 * Spin-summed density matrices of C (host outputs): gamma[p][q] = g1[0] + g1[1]
 * (n^2) and Gamma[p][q][r][u] = sum over both spins of
 * <C| a+_p a+_r a_u a_q |C> (n^4; NULL skips it). Same conditions as casci_rdm.
 */
int casci_rdm_spin_free(casci_ctx* ctx, const double* C, int mem, double* gamma, double* Gamma);

/*
 * <S^2> of a normalised FP64 CI vector C (Na x Nb): S^2 = Sz^2 + Sz + S- S+.
 * Result to host *s2.
 */
int casci_spin_square(casci_ctx* ctx, const double* C, double* s2, int mem);

typedef struct {
    int max_iter;           /* 0 -> 200 */
    int m_max;              /* subspace size before collapse; 0 -> max(8, 8*nroots) */
    int precond;            /* CASCI_PRECOND_* */
    int spin;               /* CASCI_SPIN_* */
    int ab_prec;            /* alpha-beta arithmetic of the correction vectors (CASCI_F64/F32/BF16).
                               F32/BF16: mixed precision -- at every collapse the sigma of the
                               current Ritz vectors is recomputed in FP64, and convergence is only
                               accepted on FP64 sigma (a low-precision 'converged' triggers that
                               refinement first) */
    double refine_rnorm;    /* > 0: every sigma in FP64 once max residual < this; also after 40
                               iterations without halving the best residual (<= 0: no threshold) */
    double r_tol;           /* residual threshold; <= 0 -> max(1e-6, sqrt(tol)/10) */
    double s2_penalty;      /* lambda of H + lambda S^2 for CASCI_SPIN_SINGLET (0 -> 1 Eh); < 0: no
                               penalty, the lowest roots of even transposition parity (S = 0, 2, ...) */
    const double* guess;    /* optional [nguess][Ndet] FP64 start vectors (host or device) */
    int nguess;
    int guess_mem;
    int verbose_history;    /* reserved, set to 0 */
    /* optional, called once per iteration on the calling thread with the
       current Ritz values, residual norms and wall time since the call began */
    void (*progress)(void* user, int iteration, int nroots, const double* theta,
                     const double* rnorm, double wall_ms);
    void* progress_user;
    int graph;              /* 1: replay each sigma build from a captured HIP graph (one launch
                               per build; the vector is staged through a context buffer) */
    int buffer_roots;       /* roots followed above the requested ones (they keep a higher state
                               from replacing the highest requested root): 0 -> 1, < 0 -> none */
} casci_davidson_opts;

typedef struct {
    int iterations;
    int sigma_calls;        /* vectors pushed through sigma, all precisions */
    int sigma_calls_fp64;
    int converged;          /* 1 if every root met both thresholds */
    int switch_iter;        /* iteration at which every sigma moved to FP64 (-1 = never/FP64 only) */
    int mlp_fallbacks;      /* learned corrections replaced by the Olsen fallback */
    int refinements;        /* mixed precision: restarts with FP64 sigma of the Ritz vectors */
    double residual[CASCI_MAX_ROOTS];
    double s2[CASCI_MAX_ROOTS];
    double time_total_ms;   /* wall time of the call */
    double time_sigma_ms;   /* device time spent in sigma builds */
    double time_setup_ms;   /* operator/diagonal preparation inside the call */
    /* optional per-iteration history, caller-owned, [hist_len][nroots] */
    double* hist_energy;
    double* hist_residual;
    double* hist_time_ms;   /* [hist_len]: wall time from the start of the call */
    int hist_len;
} casci_davidson_info;

/*
 * davidson: lowest nroots (1..CASCI_MAX_ROOTS) eigenpairs of H in the
 * (nalpha, nbeta) determinant space (or its S = 0 part), ascending, by the
 * Davidson-Liu method (Sec. II.A.1). Convergence: every root has
 * |Delta theta| < tol between iterations and residual norm < r_tol.
 * energies: host [nroots]. vectors: optional [nroots][Ndet] FP64 (host or
 * device per mem), normalised, phase: largest-|c| entry positive.
 * opts and info may be NULL. Returns CASCI_OK, or CASCI_NOCONV (> 0) with
 * the last Ritz pairs filled in.
 */
int casci_davidson(casci_ctx* ctx, int nroots, double tol, const casci_davidson_opts* opts,
                   double* energies, void* vectors, int mem, casci_davidson_info* info);

/*
 * batch_davidson: independent solves of `count` contexts (each with its own
 * strings, integrals and stream; no context may appear twice), nroots
 * roots each, with the same tol and options, run concurrently on up to
 * nthreads host threads (<= 0: min(count, 16)); their device work overlaps
 * on the contexts' streams. This is the many-small-active-spaces workload
 * (Sec. II.A.1's solver applied to a set of CASCI problems of uneven size):
 * set opts->graph = 1 to replay every sigma build from a captured graph.
 * energies: host [count][nroots]; infos: optional [count]. A progress
 * callback in opts is called from the worker threads. Returns the first
 * negative status of any solve (its message in that context), else
 * CASCI_NOCONV if any solve did not converge, else CASCI_OK.
 */
int casci_batch_davidson(casci_ctx* const* ctxs, int count, int nroots, double tol,
                         const casci_davidson_opts* opts, double* energies, casci_davidson_info* infos,
                         int nthreads);

/*
 * Autotuner choice of the same-spin gather for this context's string space:
 * out[0] / out[1] = strip width code of the FP64 and of the FP32-input
 * gather: 16, 32 or 64 lanes per gathered entry with one column each, 128
 * (64 lanes with two adjacent columns each), or L * 100 + V for L lanes per
 * entry with V adjacent columns each (1602, 3202; FP32 input also 1604, 3204,
 * 6404), or 99: row blocks of 32 (or 16) strings whose union of neighbour
 * rows is staged in LDS (fewer than 65536 strings); 0 until the first sigma
 * build in that precision. The code changes only the speed: every width sums
 * in the same order, so sigma is bitwise the same whichever is chosen, with
 * one exception: in BF16 builds width 99 sums in FP32 (relative difference
 * ~1e-6, far below the BF16 alpha-beta error), the others in FP64.
 */
int casci_get_tuning(casci_ctx* ctx, int* out);

/* Override the autotuner: strip width code (16, 32, 64, 128, 1602, 3202, 1604,
 * 3204, 6404 or 99 as above; 0 = autotune) of the FP64 and of the FP32-input gather
 * for this context (a vector width the row stride does not allow falls back
 * to one column per lane). */
int casci_set_tuning(casci_ctx* ctx, int f64_lpe, int f32in_lpe);

/*
 * Layout of the FP64 alpha-beta contraction (eq. (hamiltonian), the
 * opposite-spin two-electron term), per pair set: out[0] for pair rows r <= s
 * (integrals with 8-fold symmetry, no S^2 penalty), out[1] for all ordered
 * pairs. Code 10 MT + split: MT = 1 or 2 sixteen-row M tiles per wave, the
 * sigma row of an alpha string in split (1..4) times the fewest LDS chunks
 * that fit; 0 until the first FP64 build with that pair set, whose autotuner
 * times the layouts that have a kernel variant for the shape on the first
 * eighth of the alpha strings and keeps the fastest for (device, norb,
 * nalpha, nbeta, pair set) in this process. Every layout gives bitwise the
 * same sigma (fixed-point sums).
 */
int casci_get_ab_layout(casci_ctx* ctx, int* out);

/* Override the FP64 alpha-beta layout of pair set pairs (0 or 1, as above)
 * for this context: code 0 (autotune at the next build) or 10 MT + split with
 * MT 1..2 and split 1..4; CASCI_E_ARG otherwise. A layout with no kernel
 * variant for the shape makes the next FP64 build fail (CASCI_E_DEVICE, the
 * message names the missing variant). */
int casci_set_ab_layout(casci_ctx* ctx, int pairs, int code);

/*
 * Layout check for bindings: out[0..5] = sizeof(casci_davidson_opts),
 * sizeof(casci_davidson_info), offsetof(opts, progress), offsetof(info,
 * residual), offsetof(info, hist_energy), offsetof(info, hist_len). n >= 6.
 * Works on a validate-only build (no device needed).
 */
int casci_abi_layout(int64_t* out, int n);

/*
 * Dense symmetric eigensolver of the Davidson solver's small projected
 * matrices (Rayleigh-Ritz step, start-space block), host memory only, no
 * device needed: Householder tridiagonalisation, then implicit QR with
 * Wilkinson shifts. A: n x n row-major, symmetric (the lower triangle is
 * read). w[n]: eigenvalues ascending. Z[n x n] row-major: column j is the
 * unit eigenvector of w[j]. Returns CASCI_E_ARG (n < 0 or a null pointer),
 * CASCI_E_NONFINITE, or CASCI_E_UNSUPPORTED if the iteration did not
 * converge. Costs O(n^3); meant for n up to a few hundred.
 */
int casci_sym_eig(const double* A, int n, double* w, double* Z);

/*
 * Tile pairs of the S + p S^T combination of the transposition-parity sigma
 * (host computation of the same mapping the kernel's workgroups use): for
 * k = k0 .. k0+count-1, out[2(k-k0)] = bi and out[2(k-k0)+1] = bj of the k-th
 * pair bi <= bj < nb in row-by-row order. Host memory only, no device.
 * CASCI_E_ARG for nb < 1, count < 0, a null out or k outside [0, nb(nb+1)/2).
 */
int casci_tile_pairs(int64_t nb, int64_t k0, int64_t count, int64_t* out);

/*
 * Row-blocked tables of a same-spin operator (the form the SS_BLOCKED gather
 * of the alpha-alpha / beta-beta terms of eq. (hamiltonian) reads), built on
 * the host exactly as the library builds them, for checking without a
 * device. Input: N < 65536 rows of r >= 2 entries, int32 columns (entry 0 the
 * diagonal, then strictly ascending) and FP64 values; R = 16 or 32 rows per
 * block. sizes[0..3] = union entries, groups, group-offset entries, blocks
 * (all 0 when a union needs more than 127 chunks of 64 rows or a row more
 * than 65535 groups). Outputs may be null (sizes only): uni[sizes[0]]
 * (uint16, the sorted union of each block, concatenated), binfo[4 blocks]
 * (union offset, union size, group-offset offset, chunks), goff[sizes[2]]
 * (per block [R][chunks + 1] first group of each chunk relative to the row),
 * rbase[N] (first group of each row), goffs / gvals [4 sizes[1]] (per group
 * the LDS byte offsets (union position mod 64) x 512 and the FP64 values,
 * slots outside the chunk 0). CASCI_E_ARG on bad sizes or columns.
 */
int casci_ss_block_tables(int64_t N, int r, const int32_t* col, const double* val, int R, int64_t* sizes,
                          uint16_t* uni, int32_t* binfo, uint16_t* goff, int32_t* rbase, uint32_t* goffs,
                          double* gvals);

/* ------------------------------------------------------------------------
 * Learned Davidson preconditioner (CASCI_PRECOND_MLP). A per-determinant
 * network 8 -> 64 -> 64 -> 1 (tanh, FP32) predicts the correction vector
 * from features of the determinant and of the current Ritz pair (theta, x,
 * r = H x - theta x, d = H_II, N determinants):
 *   f0 = tanh((d-theta)/4), f1 = asinh(r_I sqrt(N)/|r|), f2 = asinh(x_I sqrt(N)),
 *   f3 = asinh(-r_I/(d-theta) sqrt(N)/|r|), f4/f5 = alpha/beta electrons outside
 *   the aufbau orbitals / max(1, min(n_e, n-n_e)), f6 = open-shell fraction
 *   popcount(Ia^Ib)/n, f7 = tanh((d - min_I H_II)/4).
 * Parameters (CASCI_MLP_NPARAM floats): W1[8][64] (input-major), b1[64],
 * W2[64][64], b2[64], W3[64], b3. A non-finite or vanishing learned
 * correction falls back to the Olsen correction (counted in
 * casci_davidson_info.mlp_fallbacks).
 * ---------------------------------------------------------------------- */
#define CASCI_MLP_NPARAM 4801

/* Copy n = CASCI_MLP_NPARAM parameters in (host or device); resets the Adam moments. */
int casci_mlp_set_params(casci_ctx* ctx, const float* params, int64_t n, int mem);

/* Copy the current parameters to host out[CASCI_MLP_NPARAM]. */
int casci_mlp_get_params(casci_ctx* ctx, float* out);

/* Network outputs Y[N] for feature rows X[N][8] (host or device). */
int casci_mlp_forward(casci_ctx* ctx, const float* X, int64_t N, float* Y, int mem);

/*
 * Mean squared error L = (1/N) sum (y_i - T_i)^2 over all N rows and its
 * gradient with respect to the parameters (host grad[CASCI_MLP_NPARAM] and
 * *loss, either may be NULL). Summation order is fixed (reproducible).
 */
int casci_mlp_loss_grad(casci_ctx* ctx, const float* X, const float* T, int64_t N, float* grad,
                        double* loss, int mem);

/*
 * Adam training (beta1 0.9, beta2 0.999, eps 1e-8) of the context's
 * parameters on rows (X, T): `epochs` passes over a seeded shuffle, mini-batch
 * `batch` (>= 64), learning rate lr. loss_hist: optional host [epochs] mean
 * training loss per epoch.
 */
int casci_mlp_train(casci_ctx* ctx, const float* X, const float* T, int64_t N, int epochs, int batch,
                    float lr, uint64_t seed, double* loss_hist, int mem);

/*
 * Training data from the method itself: runs casci_davidson(nroots, tol, opts)
 * and, at every iteration and for every root j, draws `samples` determinant
 * indices (seeded) and writes their features F[row][8] and targets
 * T[row] = (s x*_j - x_j)_I sqrt(N)/|s x*_j - x_j| (s = sign of x*_j . x_j),
 * with x* = xstar (device, [nroots][Ndet], the converged vectors). F, T are
 * device buffers of max_rows rows; *nrows = rows written. Returns the
 * Davidson status.
 */
int casci_mlp_collect(casci_ctx* ctx, int nroots, double tol, const casci_davidson_opts* opts,
                      const double* xstar, int samples, uint64_t seed, float* F, float* T,
                      int64_t max_rows, int64_t* nrows);

/*
 * Features F[m][8] (host) of the determinants idx[0..m) (host) for the Ritz
 * pair (theta, x) whose sigma vector is sx (x, sx: device FP64 [Ndet]).
 * CASCI_E_ARG if an index lies outside [0, Ndet) (checked before any device work).
 */
int casci_mlp_features(casci_ctx* ctx, const double* x, const double* sx, double theta,
                       const int64_t* idx, int m, float* F);

/*
 * Profiling aid: on != 0 resets and starts accumulating the device time of
 * each part of every sigma build on this context (sigma and davidson),
 * measured with HIP events recorded on the context stream between the
 * parts; each build then waits for its last event. on = 0 stops.
 */
int casci_profile_enable(casci_ctx* ctx, int on);

/*
 * out[0..15]: out[0..5] for sigma builds with FP64 alpha-beta arithmetic and
 * out[6..11] for low-precision builds, each = {alpha-alpha gather ms (with the
 * conversions of C if any), beta-beta ms (transposes + gather, or nothing
 * with parity), alpha-beta contraction ms, final combination ms, whole build
 * ms, number of builds}; out[12] = the conversions of C alone in the
 * low-precision builds of FP64 vectors (included in out[6]); out[13..15] = 0.
 * All parts run in order on the context's stream. Accumulated since
 * casci_profile_enable(ctx, 1).
 */
int casci_profile_read(const casci_ctx* ctx, double* out);

#ifdef __cplusplus
}
#endif

#endif /* CASCI_H */

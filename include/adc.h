/*
 * adc.h -- C ABI of the MI355X sigma-build library for CD-based relativistic
 * ADC(2)/ADC(3)/ADC(2)+x(3) (EE, IP, EA).
 *
 * The library solves the Hermitian secular problem M X = X Omega, X^H X = 1
 * (Section 2.1, eq. 10) for the k algebraically lowest roots, where M is the
 * ISR secular matrix in Moller-Plesset partitioning truncated per block by
 * perturbation order (eq. 11) and, for the x-scaled variant (Section 2.1,
 * sm-ADC), M(x) = M_ADC(2) + x (M_ADC(3) - M_ADC(2)).  Two-electron integrals
 * enter only through complex Cholesky vectors, <pq||rs> = sum_Q (L^Q_pr L^Q_qs
 * - L^Q_ps L^Q_qr) (Section 2.5, eq. 43); the four-external <ab||cd> are
 * never stored, they are rebuilt batch-wise from L on every sigma build.  The
 * three-external class <ia||bc> (o v^3 elements) is stored in device memory,
 * as are all classes with two or more occupied indices.
 *
 * Conventions
 *   - complex numbers are interleaved (re, im) float64 pairs ("c128");
 *   - spinor index order: occupied 0..o-1, then virtual o..o+v-1;
 *   - L is c128 [n_chol][n][n] row-major, n = o+v, Hermitian in (p,q) for
 *     every Q (the MO transform of real AO Cholesky vectors, eq. 42);
 *   - packed ISR vectors (occupied indices first, pairs i<j, a<b in
 *     lexicographic order):
 *        EE: [ (i,a) i-major                 | ((i<j),(a<b)) pair-major ]
 *        IP: [ i                             | ((i<j), a) ]
 *        EA: [ a                             | (i, (a<b)) ]
 *     The basis states are a+_a a_i, a+_a a_i a+_b a_j (EE), a_i, a+_a a_i a_j
 *     (IP), a+_a, a+_a a+_b a_j (EA) applied to the MP ground state and
 *     orthonormalised as in Section 2.1;
 *   - eigenvalues are E_n(N') - E_0(N) in hartree, ascending.
 *
 * Return codes: 0 = OK, +1 = ADC_NOT_CONVERGED (a warning: outputs are filled
 * and converged[r] is 0 for the affected roots), negative = error.  No C++
 * exception crosses this interface; the library never frees caller memory.
 * One handle must not be used from two host threads at once; distinct handles
 * are independent.
 */
#ifndef ADC_H
#define ADC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum adc_kind { ADC_EE = 0, ADC_IP = 1, ADC_EA = 2 };

/* Arithmetic of the sigma build.  ADC_FP64 runs every contraction in FP64;
 * ADC_FP32 runs the large trial-vector contractions (ladder, ring, coupling)
 * on FP32 MFMA with FP32 accumulation; ADC_SPLIT_BF16 splits each FP32
 * operand into bf16 hi + lo and accumulates three bf16 MFMA products in FP32.
 * M11, the diagonal and all Davidson algebra always stay FP64. */
enum adc_precision { ADC_FP64 = 0, ADC_FP32 = 1, ADC_SPLIT_BF16 = 2 };

enum adc_status {
  ADC_OK = 0,
  ADC_NOT_CONVERGED = 1,
  ADC_ERR_INVALID_ARG = -1,
  ADC_ERR_NONFINITE_INPUT = -2,
  ADC_ERR_NOT_HERMITIAN = -3,
  ADC_ERR_OUT_OF_MEMORY = -4,
  ADC_ERR_HIP = -5,
  ADC_ERR_UNSUPPORTED = -6,
  ADC_ERR_SCRATCH = -7
};

/* One problem (instance).
 *   kind      ADC_EE / ADC_IP / ADC_EA
 *   n_occ     o >= 1, n_vir v >= 2, n_chol N >= 1, n_roots k >= 1
 *   eps       host float64 [o+v], occupied first, in hartree; copied
 *   L         c128 [N][n][n] (see above); host memory (copied to the device
 *             at adc_init) or, with L_on_device = 1, a device pointer that is
 *             borrowed and must stay valid until adc_free
 *   x         scaling of the third-order part; 1 = ADC(3), 0 = ADC(2); any
 *             finite value is accepted */
typedef struct adc_problem {
  int kind;
  int n_occ, n_vir, n_chol, n_roots;
  const double* eps;
  const void* L;
  int L_on_device;
  double x;
} adc_problem;

/* Options (zero-initialised fields take the defaults in brackets).
 *   precision     default arithmetic of adc_sigma / adc_davidson [ADC_FP64]
 *   conv_tol      residual norm threshold of the Davidson solver [1e-7]
 *   max_iter      Davidson iterations [200]
 *   max_subspace  subspace size before collapse to 2k [6k; at least 3k,
 *                 at most dim]
 *   refine_fp64   mixed precision only: 0 or 1 = iterate in the reduced
 *                 precision to a residual of 1e-4 (or conv_tol if larger),
 *                 or, once the largest residual is below 1e-6 max|omega|,
 *                 until it has not come down by 10% for 15 iterations (the
 *                 reduced precision leaves a residual floor of about 1e-7
 *                 |omega|), then restart from the Ritz
 *                 vectors in FP64 until the FP64 residual meets conv_tol
 *                 [0 = 1]; -1 = no FP64 restart: the reduced-precision sweep
 *                 itself iterates to conv_tol and the reported residuals are
 *                 its own
 *   stream        hipStream_t to enqueue on; NULL = a library-owned stream
 *   mem_budget    bytes of device workspace: sizes the <ab||cd> batches,
 *                 the largest temporary copy a contraction may make before it
 *                 is split into pieces, and how many trial vectors one pass
 *                 of the unpacked-doubles terms takes, and a quarter of it
 *                 the packed <ab||cd> rows contracted at once [0 = 4 GiB
 *                 batches, 8 GiB copies, 16 GiB per pass, and in split-bf16
 *                 all packed rows at once when they take at most 16 GiB];
 *                 results do not depend on it beyond rounding
 *   verbose       1 = one line per Davidson iteration on stderr; 2 = also
 *                 one line per GEMM launch (shape, tile, split, output map)
 *   n_streams     several instances: number of lanes (device streams, each
 *                 with its own workspace) the instances are spread over,
 *                 most expensive first [min(n_problems, 4)]; lane 0 is
 *                 `stream`, the others are library-owned non-blocking streams
 *                 of default priority
 *   graphs        inside adc_davidson: 1 = replay each small instance's
 *                 sigma build from a captured hipGraph, and run the rest of
 *                 each iteration on the device (Gram matrix, the subspace
 *                 eigenproblem in one workgroup, Ritz vectors, residuals,
 *                 convergence test, preconditioner with Olsen's correction,
 *                 collapse, orthonormalisation of the new directions), from
 *                 one captured hipGraph per subspace size, with one small
 *                 device-to-host report per iteration; 2 = the same device
 *                 iteration launched kernel by kernel, sigma builds eager;
 *                 0 = host-driven iteration (subspace eigenproblem on the
 *                 host) [0].  Root following, and subspaces of more than
 *                 256 vectors, always run host-driven.
 *   autotune      1 = time the tile and split-K candidates of every GEMM
 *                 shape class once and keep the fastest [0]
 *   tune_cache    path of a text file of tuned GEMM choices (one shape class
 *                 per line) or NULL [NULL]: read at adc_init when it exists,
 *                 so that with autotune on the shape classes it holds are not
 *                 timed again; written back (every class tuned in the
 *                 process) at adc_free when autotune is on; a file that
 *                 cannot be read is ignored
 *   deterministic 1 = every tile and split-K choice comes from the fixed
 *                 cost model (autotune and tune_cache are ignored), so that
 *                 repeated calls with the same inputs and options give
 *                 bitwise identical results on the same device [0]; the
 *                 library has no atomics in its arithmetic, so only timed
 *                 choices can change rounding between runs
 *   root_follow   1 = root-specific Davidson (Section 2.4, the root-specific
 *                 solver of the SS-FNS scheme) for instances given a start
 *                 block: root r is, in every iteration, the Ritz pair with the
 *                 largest overlap with start vector r (among those not taken
 *                 by an earlier root) instead of the r-th lowest; omega is
 *                 then in the order of the start vectors [0]
 *   precond       Davidson preconditioner: 0 = on the singles block the
 *                 exact (w_r - M11)^-1, from an FP64 eigendecomposition of
 *                 M11 made once at the start of each solve (rocSOLVER; only
 *                 for n1 <= 12288 and without deterministic, else the
 *                 diagonal), on the doubles the zeroth-order diagonal; 1 =
 *                 the zeroth-order diagonal throughout [0].  Olsen's
 *                 correction applies to either. */
typedef struct adc_options {
  int precision;
  double conv_tol;
  int max_iter;
  int max_subspace;
  int refine_fp64;
  void* stream;
  size_t mem_budget;
  int verbose;
  int n_streams;
  int graphs;
  int autotune;
  const char* tune_cache;
  int deterministic;
  int root_follow;
  int precond;
} adc_options;

typedef struct adc_handle adc_handle;

/* Set up n_problems >= 1 independent instances (each of any kind and size)
 * for the secular problem of Section 2.1, eq. 10 with M(x) of eq. 11 and the
 * sm-ADC scaling: validate them, copy eps (and L unless borrowed) to the
 * device and run the one-off work of every instance on the device.  That is
 * the stored antisymmetrised integral classes <ij||kl>, <ij||ka>, <ij||ab>,
 * <ia||jb>, <ia||bc>, each a sum over Cholesky vectors (Section 2.5, eq. 43);
 * the MP amplitudes t(1), t(2) (with one pass of the particle-particle ladder)
 * and the second-order singles, on which the intermediate states are built
 * (Section 2.1, the CES applied to the MP ground state); the dense singles
 * block M11 through third order with its third-order part kept separate so
 * that x scales it.
 *   problems   host array of n_problems entries (read during the call only)
 *   opts       NULL = all defaults
 *   out        receives the handle; NULL on error
 * Errors: INVALID_ARG (shapes, NULL pointers, n_problems < 1, an option out
 * of its documented range: negative or non-finite conv_tol, negative max_iter
 * or max_subspace, refine_fp64 outside -1..1, an unknown precision, graphs or
 * precond value; adc_last_error names it),
 * NONFINITE_INPUT (NaN/Inf in eps, x or L), NOT_HERMITIAN (max |L^Q - L^Q^H| >
 * 1e-12 max |L^Q| for some Q; L^Q is Hermitian as the MO transform of real AO
 * Cholesky vectors, eq. 42), OUT_OF_MEMORY, HIP_ERROR.  A borrowed device L
 * is checked on the device, a host L on the host.  On error *out is NULL and
 * nothing is leaked.  Synchronous. */
int adc_init(const adc_problem* problems, int n_problems, const adc_options* opts,
             adc_handle** out);

/* Sizes n1 (singles) and n2 (doubles) of the intermediate-state basis of
 * instance inst (Section 2.1, the CES classes of each kind), packed as
 * described above; dim = n1 + n2.  Errors: INVALID_ARG. */
int adc_dims(const adc_handle* h, int inst, long long* n1, long long* n2);

/* The sigma build S = M(x) Y for k packed c128 vectors: the product of the
 * secular matrix of Section 2.1 (eq. 10; blocks by order as in eq. 11, the
 * third-order part scaled by x as in sm-ADC) with trial vectors, as the
 * Davidson solver of eq. 10 needs it.  The four-external <ab||cd> are
 * rebuilt from L batch by batch on every call (Section 2.5, eq. 43 and the
 * on-the-fly generation of the four-external integrals), never stored.
 * Y and S are device arrays [k][dim], must not alias, and stay owned by the
 * caller.  precision < 0 uses the handle's default.  Enqueued on the
 * handle's stream (asynchronous).  Workspace comes from the handle's device
 * pool (allocated on first use and kept).  Errors: INVALID_ARG, HIP_ERROR,
 * OUT_OF_MEMORY. */
int adc_sigma(adc_handle* h, int inst, const void* Y, void* S, int k, int precision);

/* The sigma build of adc_sigma (same arguments, same result) without any
 * device allocation, for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Every
 * temporary of the build comes from one fixed device array of 128 MiB per
 * GPU (held from the library's load until the process ends); the build plans
 * its passes, <ab||cd> batches and temporary copies for that size, times no
 * GEMM variant, and makes no persistent cache entry (it still reads the
 * handle's existing ones).  The handle's own state (integral classes,
 * amplitudes, M11) was allocated by adc_init.
 * A request that certainly needs more than the array (its doubles
 * accumulators or one <ab||cd> block of one a alone) is rejected with
 * ADC_ERR_SCRATCH before anything is enqueued.  A build that runs out of the
 * array part-way also returns ADC_ERR_SCRATCH, after the work already
 * enqueued has finished (S is then undefined), and later requests of that
 * precision with at least as many vectors are rejected up front.
 * Calls on one GPU share its array and it keeps the last call's contents:
 * calls that overlap on one GPU (any handle, any stream) race, so serialise
 * them; nothing relies on the array starting at zero.
 * Errors: INVALID_ARG, SCRATCH, HIP_ERROR (also when the array's address
 * could not be taken on this device). */
int adc_sigma_noalloc(adc_handle* h, int inst, const void* Y, void* S, int k, int precision);

/* Block Davidson for the n_roots lowest eigenpairs of every instance
 * (Section 2.1, eq. 10: M X = X Omega, X^H X = 1, with sigma builds as
 * above; the paper's Davidson settings are not printed, so the guess,
 * preconditioner and convergence rules are this library's).  The
 * per-root outputs are concatenated over the instances in order (instance i
 * starts at the sum of n_roots of instances < i); the lanes solve their
 * instances concurrently.
 *   guess        NULL, or guess[inst] = NULL or device c128 [n_roots][dim]
 *                start vectors (resume); when they span fewer than n_roots
 *                directions the rest is filled with the default unit-vector
 *                guesses outside their span (INVALID_ARG if that fails)
 *   omega        host float64 [sum n_roots], ascending per instance, hartree
 *   vecs         NULL, or vecs[inst] = NULL or device c128 [n_roots][dim]
 *                output Ritz vectors
 *   resnorm      host float64 [sum n_roots]   final FP64 residual norms
 *   iters        host int [n_problems]        iterations used
 *   converged    host int [sum n_roots]       1 if the root met the criteria
 * Subspace algebra (Gram matrix, Ritz vectors, residuals, norms,
 * preconditioner, orthogonalisation) runs in FP64 device kernels; the small
 * subspace eigenproblem runs on the host (or, with graphs, on the device);
 * with precond = 0 each solve starts with one FP64 eigendecomposition of
 * the singles block M11 on the device.  Synchronous.  Returns
 * ADC_NOT_CONVERGED if any root missed the criteria, ADC_ERR_NONFINITE_INPUT
 * if a subspace matrix holds NaN or Inf (e.g. from a non-finite guess). */
int adc_davidson(adc_handle* h, const void* const* guess, double* omega, void* const* vecs,
                 double* resnorm, int* iters, int* converged);

/* One term of the sigma build, for per-term checks and timing:
 *   ADC_TERM_ALL      same as adc_sigma
 *   ADC_TERM_LADDER   S = x * (particle-particle ladder) Y: the doubles part
 *                     sum_{c<d} <ab||cd> Y_..cd, the <ab||cd> built batch-wise
 *                     from L (Section 2.5, eq. 43, generated on the fly), the
 *                     term part of the first-order doubles block of eq. 11
 *                     (EE and EA; singles part of S set to zero)
 * Same argument rules as adc_sigma.  Errors: INVALID_ARG, UNSUPPORTED (the
 * term does not exist for the kind), HIP_ERROR. */
enum adc_term { ADC_TERM_ALL = 0, ADC_TERM_LADDER = 1 };
int adc_sigma_term(adc_handle* h, int inst, int term, const void* Y, void* S, int k, int precision);

/* Vector-Jacobian product of the sigma build.  For the real functional
 *     f(L, x) = Re sum_z Sbar_z^H M(L, x) Y_z
 * with fixed packed vectors Y, Sbar (device c128 [k][dim], caller-owned):
 *   dL   device c128 [n_chol][n][n] (caller-owned, overwritten), the gradient
 *        G = df/dRe L + i df/dIm L projected onto Hermitian L^Q,
 *        (G + G^H)/2 per Q; NULL skips it.  Only Hermitian perturbations of
 *        the Cholesky vectors keep M Hermitian (Section 2.1, eq. 10; eq. 42).
 *   dx   host double, df/dx = f(x+1) - f(x) (M is affine in x); NULL skips.
 * With Sbar = Y = a normalised eigenvector y_r this is the eigenvalue
 * gradient d omega_r = y_r^H dM y_r (Hellmann-Feynman).  The gradient with
 * respect to Y is adc_sigma applied to Sbar (M is Hermitian).
 * The one-off work of adc_init and the sigma build are recomputed on the
 * device with their intermediates kept, then differentiated in reverse,
 * every reverse rule in the arithmetic of its forward operation: the one-off
 * part in FP64 (as in adc_init), the sigma part in the handle's default
 * precision (FP64, FP32 or split-bf16 contractions), with every gradient
 * accumulated in complex128; dx is formed from two FP64 builds whatever the
 * precision.  The first call on an instance keeps its recorded one-off part
 * (with every buffer it wrote) until adc_free, so later calls record and
 * differentiate only the sigma build on top of it; the kept part reflects L
 * as the first call read it.  The <ab||cd> gradient blocks of the
 * particle-particle ladder are formed per batch of a from L and never stored
 * whole.  Device memory: about twice that of adc_init plus one workspace
 * batch, the one-off part staying allocated between calls.  Synchronous.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, HIP_ERROR (after an error the kept
 * part is dropped and the next call records it again). */
int adc_sigma_backward(adc_handle* h, int inst, const void* Sbar, const void* Y, int k,
                       void* dL, double* dx);

/* ISR one-particle properties of EE states (Section 2.2): for the k packed
 * vectors Y (device c128 [k][dim], each normalised by the library first)
 *   tdm  = rho^{0->K}_pq = sum_I conj(Y_IK) f^I_pq,  f^I_pq = <Psi~_I|c+_p c_q|Psi_0>
 *          through first order (the reading: the paper fixes no order);
 *   rho  = rho^K_pq = Y_K^* g(0) Y_K + rho_GS(2)_pq, the zeroth-order ISR
 *          density of the state plus the second-order ground-state
 *          correlation density (the shifted form Y^* G Y + D_0 with D_0 through
 *          second order);
 * both device c128 [k][n][n] (caller-owned, n = o + v, element [p][q] for
 * c+_p c_q, occupied spinors first), each optional.  With a one-particle
 * operator d (device c128 [n][n]) the library also returns D_K = sum_pq d_pq
 * rho^K_pq (dk) and T_{0->K} = sum_pq d_pq rho^{0->K}_pq (tk), host float64
 * [2k] as (re, im) pairs.  FP64 device contractions.  Synchronous.
 * Errors: INVALID_ARG (k < 1, dk or tk without d), UNSUPPORTED (not EE),
 * OUT_OF_MEMORY, HIP_ERROR. */
int adc_properties(adc_handle* h, int inst, const void* Y, int k, void* rho, void* tdm, const void* d, double* dk,
                   double* tk);

/* Frozen natural spinors of instance inst (Section 2.4, eqs. 25-30): the
 * virtual-virtual density D_ab = 1/2 sum_{cij} <ac||ij><ij||bc> /
 * (e_ij^ac e_ij^bc) (eq. 25), plus, when X is given, the state density of X
 * through the zeroth-order intermediate states, D_ab += <X| a+_b a_a |X>
 * (eq. 31, state-specific FNS; EE and EA only); its eigenvectors (natural
 * spinors, eq. 26) with occupation >= eta_crit kept (eq. 27); the Fock block
 * in that basis diagonalised (eqs. 28-29); B = V~ Z~ (eq. 30).  The problem is
 * then given in the truncated basis: virtual spinor a' = sum_a a B_aa', and the
 * Cholesky vectors follow (eq. 42 with the coefficients C B).
 *   X        NULL, or device c128 [dim] a vector of the instance (normally an
 *            ADC(2) eigenvector) for the state-specific density
 *   eta_crit occupation threshold (finite)
 *   n_vir    host: v', the number of kept virtual spinors (>= 2)
 *   eps_out  host float64 [o + v]: the occupied energies, then the v'
 *            semicanonical virtual energies (ascending)
 *   L_out    device c128, room for [N][o+v][o+v]; receives [N][o+v'][o+v']
 *            (Hermitian per Q), ready for adc_init with n_vir = v'
 *   eta_out  NULL or host float64 [v]: the occupations, descending
 *   B_out    NULL or device c128, room for [v][v]; receives B as [v][v']
 *   X_out    NULL or device c128, room for X's size: X in the truncated basis
 *            (every virtual index contracted with conj(B), packed for v'),
 *            the start vector of the truncated problem
 * The v x v and v' x v' Hermitian eigenproblems run on the host (cyclic
 * Jacobi); the density, the vector and Cholesky transforms are device GEMMs
 * in FP64.  Synchronous.  Errors: INVALID_ARG (NULL outputs, eta_crit keeping
 * fewer than two spinors), UNSUPPORTED (X given for an IP instance),
 * OUT_OF_MEMORY, HIP_ERROR. */
int adc_fns(adc_handle* h, int inst, const void* X, double eta_crit, int* n_vir, double* eps_out, void* L_out,
            double* eta_out, void* B_out, void* X_out);

/* One-step pivoted Cholesky of the electron-repulsion matrix (Section 2.5,
 * eq. 41 and the one-step procedure): V is the symmetric positive
 * semidefinite matrix (mu nu|kappa lambda) over m composite indices (for
 * instance the pairs mu <= nu), device float64 [m][m] row-major, read only.
 * Vector k is made at the largest remaining diagonal element d_p of
 * V - sum_{q<k} L_q L_q^T (lowest index among equal ones):
 * L_k[i] = (V[p][i] - sum_{q<k} L_q[i] L_q[p]) / sqrt(d_p); the procedure ends
 * when d_p < tau (or d_p <= 0) or after max_vec vectors, so that
 * V ~ sum_k L_k L_k^T with every remaining diagonal element below tau.
 *   L       device float64 [max_vec][m] (caller-owned); rows >= n_vec unset
 *   pivots  host int [max_vec]: p of each vector
 *   n_vec   host: number of vectors made
 *   stream  hipStream_t (NULL = the default stream)
 * Temporaries (the remaining diagonal, the step state) are allocated and
 * freed inside the call.  Synchronous.  Errors: INVALID_ARG (m < 1 or
 * >= 2^31, tau < 0 or not finite, NULL outputs), NONFINITE_INPUT (a
 * non-finite diagonal element), OUT_OF_MEMORY, HIP_ERROR. */
int adc_cholesky(const double* V, long long m, double tau, int max_vec, double* L, int* pivots, int* n_vec,
                 void* stream);

/* The Cholesky vectors in the molecular spinor basis (Section 2.5, eq. 42):
 * L^P_pq = sum_{mu nu} conj(C_mu p) L^P_mu nu C_nu q, Hermitian in (p, q)
 * for real symmetric L^P_mu nu.
 *   Lp    device float64 [n_vec][n_ao (n_ao + 1) / 2]: each vector over the
 *         pairs mu <= nu in row-major upper-triangle order (as made by
 *         adc_cholesky on a V over those pairs), read as symmetric
 *   C     device c128 [n_ao][n_mo] MO coefficients
 *   Lmo   device c128 [n_vec][n_mo][n_mo] (caller-owned): the L of
 *         adc_problem for n_mo = o + v spinors ordered occupied first
 * FP64 complex GEMMs on the matrix cores.  Synchronous.  Errors:
 * INVALID_ARG, OUT_OF_MEMORY, HIP_ERROR. */
int adc_cholesky_mo(const double* Lp, int n_vec, int n_ao, const void* C, int n_mo, void* Lmo, void* stream);

/* Milliseconds spent in adc_init on the device (one-off work). */
double adc_init_ms(const adc_handle* h);

/* Release every library allocation of the handle.  NULL is accepted. */
void adc_free(adc_handle* h);

/* Static message for a status code. */
const char* adc_strerror(int code);

/* Detail of the calling thread's most recent failed call on a handle
 * (adc_init .. adc_sigma_backward): the check or step that failed (an
 * argument rejected up front names its entry point, "adc_sigma: ...") and,
 * for HIP errors, the runtime's message; "" when that call succeeded.  The
 * text stays valid until the thread's next such call. */
const char* adc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ADC_H */

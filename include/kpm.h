/*
 * kpm.h -- C ABI of the MI355X (gfx950) library for the stochastic
 * Chebyshev-moment ("kernel polynomial") typicality method of
 * H. Schlueter, F. Gayk, H.-J. Schmidt, A. Honecker, J. Schnack,
 * "Accuracy of the typicality approach using Chebyshev polynomials",
 * arXiv:2104.13218 (cited below as "the paper").
 *
 * Problem statement (the paper, Sec. II and Sec. III): spin-1/2 Heisenberg
 * Hamiltonians H = sum_b J_b s_i . s_j given by a bond list on N sites, split
 * into S^z sectors (Sec. II, after Eq. (3), and the sector sum below Eq. (9));
 * parameters: expansion order (moment count M), scaling parameter eps of
 * Eq. (5), number of random vectors R of Eq. (7), kernel g_n of Eq. (8) and the
 * number of quadrature nodes (the paper's N-tilde).
 *
 * Conventions
 *  - Every function returns an int status: KPM_OK (0) or a negative KPM_E*
 *    code; kpm_strerror() names it.  On error the outputs are unspecified,
 *    nothing is leaked and the library stays usable.  No C++ exception leaves
 *    the library: a failed host allocation is KPM_ENOMEM, any other internal
 *    failure KPM_EDEVICE, and a *_workspace_size() query that fails returns 0.
 *  - Problem descriptions (kpm_problem, kpm_params, bond arrays, and host
 *    arrays marked "host") are read during the call only.
 *  - Arrays marked "device" are device pointers in the current HIP device's
 *    memory, owned by the caller.  Results are written on `stream` (a
 *    hipStream_t passed as void*, NULL = the null stream) and are complete when
 *    the call returns (every call synchronises `stream` before returning).
 *  - Workspace: device scratch comes from the caller as (d_work, work_bytes)
 *    sized by the matching *_workspace_size() query; d_work == NULL makes the
 *    library allocate and free it inside the call.  Too small a workspace is
 *    KPM_EWORKSPACE.
 *  - Layout conventions: a problem's basis is the ascending-integer order of
 *    N-bit words with n_up set bits (bit p set <=> site p is up); index = rank
 *    in the combinatorial number system.
 *  - Thread safety: calls on different streams may run concurrently.  Global
 *    state: a per-device cache of tuned launch shapes (mutex-guarded), the
 *    per-device scratch array of chebyshev_moments_noalloc (its calls on one
 *    device are serialised by a mutex), and the statistics of each host
 *    thread's last run (kpm_last_run_stats, thread-local).
 */
#ifndef KPM_H
#define KPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define KPM_OK 0
#define KPM_EINVAL (-1)     /* invalid argument (bad bond, n_up, M, ...) */
#define KPM_ENOMEM (-2)     /* device (or host) allocation failed */
#define KPM_EDEVICE (-3)    /* HIP runtime error */
#define KPM_EBOUNDS (-4)    /* |mu_n| > mu_0 (1 + 1e-6) for some vector: the
                               spectral bounds do not enclose the spectrum */
#define KPM_EWORKSPACE (-5) /* caller workspace smaller than required */
#define KPM_ETOOLARGE (-6)  /* chebyshev_moments_noalloc: the call needs more than
                               KPM_NOALLOC_MAX_BYTES of workspace */

/* ---- random vector kinds of Eq. (7) ------------------------------------- */
#define KPM_VEC_RADEMACHER 0       /* components +-1                         */
#define KPM_VEC_COMPLEX_GAUSSIAN 1 /* complex Gaussian, <r|r> = dim;         */
                                   /* stored as two real columns (Re, Im)    */
#define KPM_VEC_GAUSSIAN 2         /* real Gaussian (the paper's choice),    */
                                   /* <r|r> = dim                            */
#define KPM_VEC_BASIS 3            /* complete basis e_nu: exact traces,     */
                                   /* Eq. (6) (the paper's check of Sec. II) */

/* ---- storage precision of the recursion vectors ------------------------- */
#define KPM_FP64 0       /* float64 vectors, float64 arithmetic               */
#define KPM_FP32_STORE 1 /* float32 vectors; float64 products, sums and dots  */
#define KPM_FP32R_STORE 2 /* float32 vectors with a 16-bit residual per element
                            (6 bytes): v = hi + q 2^(e - 165), hi = float32(v)
                            rounded to nearest, e = max(1, biased exponent of
                            hi), q = rint((v - hi) 2^(165 - e)), |q| <= 2^14;
                            relative storage error <= 2^-38 (float32: 2^-24);
                            float64 products, sums and dots.  A storage form of
                            this library (the paper fixes none).  Taken by
                            chebyshev_moments and chebyshev_moments_noalloc for
                            spin-1/2 problems the slice step kernel can run
                            (KPM_EINVAL otherwise, and in every other entry
                            point) */

/* ---- kernel coefficients g_n, Eq. (8) ----------------------------------- */
#define KPM_KERNEL_NONE 0    /* g_n = 1 */
#define KPM_KERNEL_JACKSON 1 /* Jackson kernel with N_deg = M */

/* One (cluster, S^z sector) problem.  S^z = n_up - n_sites/2 >= 0 (spin 1/2). */
typedef struct {
  int32_t n_sites;       /* N, 2..32 (spin s > 1/2: 2..16 with 2s N <= 63) */
  int32_t n_up;          /* up spins, n_sites/2 <= n_up <= n_sites (2 n_up >= N); for
                            spin s (two_s >= 2): sum over sites of s + m_i = S^z + N s,
                            with 2 n_up >= 2s N (S^z >= 0) and n_up <= 2s N */
  int32_t n_bonds;       /* 0..512; i != j, 0 <= i, j < N; repeats are summed */
  int32_t cluster;       /* dense id 0.. < 65536: thermodynamic system and RNG
                            stream; problems of one cluster are its sectors */
  const int32_t* bond_i; /* host [n_bonds] */
  const int32_t* bond_j; /* host [n_bonds] */
  const double* J;       /* host [n_bonds], finite */
  double e_lo, e_hi;     /* spectral bounds E_min <= E_max of Eq. (5); NaN in
                            either => estimated by Lanczos (kpm_params) */
  int32_t two_s;         /* 2s of every site: 0 or 1 = spin 1/2; 2..7 = spin 1 .. 7/2
                            (the spin-5/2 Fe10 wheel of Sec. III.B).  H = sum_b J_b
                            S_i . S_j; the sector basis is the digit strings d_i = s + m_i
                            with the given sum in ascending value sum_i d_i (2s+1)^i.
                            Spin s > 1/2 is accepted by chebyshev_moments,
                            chebyshev_vectors, kpm_spectral_bounds, kpm_ftlm,
                            kpm_sector_eigenvalues and the thermodynamics entry points
                            (kpm_thermo, kpm_thermo_field, kpm_thermo_hybrid); the
                            gradient entry points and kpm_sector_matrix reject it with
                            KPM_EINVAL.  A call holding any spin-s problem runs every
                            problem of the call with the spin-s step kernel */
  int32_t reserved;      /* must be 0 */
} kpm_problem;

typedef struct {
  double eps;            /* Eq. (5): spectrum mapped into [-1+eps/2, 1-eps/2]; 0 <= eps < 1 */
  int32_t M;             /* moments mu_0..mu_{M-1}, M >= 2 (the paper's N_deg = M) */
  int32_t R;             /* random vectors per problem, 1..1024 (ignored for KPM_VEC_BASIS) */
  int32_t vec_kind;      /* KPM_VEC_* */
  int32_t precision;     /* KPM_FP64 | KPM_FP32_STORE */
  int32_t col_block;     /* real columns per recursion block, 0 = tuned; 1..64 */
  uint64_t seed;         /* counter-RNG seed */
  int32_t lanczos_steps; /* Lanczos steps for NaN bounds (0 => 50) */
  double bound_margin;   /* widening of Lanczos bounds, fraction of the width (>= 0) */
  int32_t autotune;      /* 0: the planner's launch shape; 1: chebyshev_moments times a few
                            recursion steps of each candidate shape (block width, step
                            kernel, tile shape, gathers in flight) the first time a
                            problem shape is seen on a device and reuses the fastest
                            (process-wide cache, mutex-guarded).  Results then differ
                            from the untuned plan by rounding only (other summation
                            order); the workspace query covers every candidate. */
} kpm_params;

/* Human-readable name of a status code (static string). */
const char* kpm_strerror(int code);

/* Sector dimension C(n_sites, n_up) (0 if out of range). Host only. */
uint64_t kpm_sector_dim(int32_t n_sites, int32_t n_up);

/* Basis enumeration (debug export).  d_states: device uint32 [C(N, n_up)],
 * written in rank order: d_states[r] = the word of rank r. 1 <= N <= 32. */
int kpm_sector_states(int32_t n_sites, int32_t n_up, uint32_t* d_states, void* stream);

/* Matrix elements of H (unscaled) for rows [row0, row0+nrows) of a sector
 * (debug export; the same device code the recursion uses).
 *  d_cols  device uint32 [nrows][max_nb]: ranks of the off-diagonal neighbours
 *          s XOR (1<<i | 1<<j) for each bond whose two bits differ, in bond order
 *  d_bond  device int32 [nrows][max_nb]: the bond index of each entry
 *          (its matrix element is J_b / 2)
 *  d_cnt   device int32 [nrows]: entries used per row (<= n_bonds)
 *  d_diag  device double [nrows]: sum_b J_b (+1/4 if bits equal, -1/4 otherwise)
 * max_nb >= n_bonds is required. */
int kpm_sector_matrix(const kpm_problem* p, int64_t row0, int64_t nrows, int32_t max_nb,
                      uint32_t* d_cols, int32_t* d_bond, int32_t* d_cnt, double* d_diag,
                      void* stream);

/* Spectral bounds for Eq. (5) (the paper estimates the ground state with
 * Lanczos, Sec. III.A.2.b): `steps` steps of float64 Lanczos without
 * reorthogonalisation from the unit-norm real Gaussian vector of RNG stream
 * r = 1023 (a +-1 start can be exactly orthogonal to an extreme eigenvector),
 * stopping early when an off-diagonal falls below 1e-12; the extreme Ritz
 * values are widened by margin*(width) on each side (a window narrower than
 * 1e-8 max(1,|E|) is widened to E -/+ 1/2).  e_lo_hi: host double [n][2]. */
int kpm_spectral_bounds(const kpm_problem* p, int32_t n, int32_t steps, double margin,
                        uint64_t seed, double* e_lo_hi, void* stream);

/* Workspace bytes for chebyshev_moments with these problems and parameters. */
size_t chebyshev_moments_workspace_size(const kpm_problem* p, int32_t n, const kpm_params* q);

/* Chebyshev moments, Eqs. (6)-(7): for each problem, with H' = (H - b)/a,
 * a = (E_hi - E_lo)/(2 - eps), b = (E_hi + E_lo)/2 (Eqs. (4)-(5)),
 *   mu_n = dim/R sum_r <r|T_n(H')|r> / <r|r>,   n = 0..M-1,
 * from the recursion v_1 = H' v_0, v_{n+1} = 2 H' v_n - v_{n-1} and the
 * doubling identities mu_2n = 2<v_n|v_n> - mu_0, mu_2n+1 = 2<v_n+1|v_n> - mu_1
 * (M/2 products).  Random vectors come from the counter-based SplitMix64
 * generator, stream (cluster << 16 | n_up << 10 | r).
 *  d_mu  device double [n][M]
 *  d_ab  device double [n][2] = (a, b), may be NULL
 * Returns KPM_EBOUNDS when some |<r|T_n|r>| exceeds <r|r>(1 + 1e-6). */
int chebyshev_moments(const kpm_problem* p, int32_t n, const kpm_params* q,
                      double* d_mu, double* d_ab, void* d_work, size_t work_bytes,
                      void* stream);

/* Size of the static per-GPU workspace array of chebyshev_moments_noalloc. */
#define KPM_NOALLOC_MAX_BYTES ((size_t)64 << 20)

/* chebyshev_moments for callers that cannot allocate device memory (serving
 * loops with a fixed memory budget, harnesses that forbid hipMalloc): the same
 * problems, parameters, results and status codes as chebyshev_moments, but no
 * device allocation of any kind (no hipMalloc/hipFree, no captured graph, no
 * events).  Differences:
 *  - Workspace: a file-scope device array of KPM_NOALLOC_MAX_BYTES bytes, one
 *    per GPU, loaded with the library and held until the process ends.  A call
 *    whose chebyshev_moments_workspace_size() exceeds it returns KPM_ETOOLARGE
 *    and writes nothing.  The array keeps the last call's contents; the call
 *    clears what must start at zero itself.
 *  - Sharing: every call on one GPU uses that GPU's one array.  Two calls that
 *    overlapped on one GPU would race, so the library serialises them with a
 *    per-GPU mutex held until the call's stream has drained (each call
 *    synchronises `stream` before it returns); concurrent callers wait.
 *  - q->autotune must be 0 (KPM_EINVAL otherwise): the planner's launch shape
 *    is used, so results equal chebyshev_moments' with autotune 0.
 *  - Recursion steps are launched one by one on `stream`; kpm_last_run_stats
 *    then reports graph_segment 0 and recursion_ms -1.
 *  d_mu  device double [n][M];  d_ab  device double [n][2] = (a, b), may be NULL.
 * Not for use under stream capture (it synchronises `stream`). */
int chebyshev_moments_noalloc(const kpm_problem* p, int32_t n, const kpm_params* q,
                              double* d_mu, double* d_ab, void* stream);

/* Workspace bytes for chebyshev_vectors (0 if the arguments are invalid). */
size_t chebyshev_vectors_workspace_size(const kpm_problem* p, const kpm_params* q,
                                        int32_t n_vec);

/* The Chebyshev vectors behind Eq. (6) for ONE problem: v_0 = the random
 * vectors of chebyshev_moments (same seeds and normalisation), v_1 = H' v_0,
 * v_{n+1} = 2 H' v_n - v_{n-1}; returns v_{n_vec} computed by the same plan
 * and step kernels as chebyshev_moments (q->M is ignored).
 *  d_out device [dim][R_cols] row-major, R_cols = R (x2 for complex vectors,
 *        Re and Im adjacent; C(N, n_up) for the complete basis), float for
 *        KPM_FP32_STORE, double for KPM_FP64
 *  d_ab  device double [2] = (a, b), may be NULL
 * Errors: KPM_EINVAL (arguments), KPM_EWORKSPACE (work_bytes too small),
 * KPM_EDEVICE (HIP error or a neighbour rank outside the sector). */
int chebyshev_vectors(const kpm_problem* p, const kpm_params* q, int32_t n_vec, void* d_out,
                      double* d_ab, void* d_work, size_t work_bytes, void* stream);

/* Thermodynamics from moments (Sec. II): kernel g_n (Eq. (8)), DOS weights
 * gamma_k at the n_nodes Gauss-Chebyshev nodes (0 => M; any n_nodes >= 1 is
 * accepted), and per cluster c and temperature T (k_B = 1,
 * g mu_B = 1):
 *   Z   = (1/n_nodes) sum_sectors W sum_k gamma_k exp(-E_k/T),  E_k = a x_k + b,
 *   E   = <E>,  C = (<E^2> - <E>^2)/T^2,  chi = (<S_z^2> - <S_z>^2)/T,
 * W = 1 for S^z = 0 sectors, 2 otherwise (the S^z < 0 mirror, Sec. II).
 *  d_mu [n][M], d_ab [n][2], d_T [n_T]: device; outputs device
 *  [n_clusters][n_T] (n_clusters = 1 + max cluster id); d_znonpos (may be NULL)
 *  flags Z <= 0 (an improper DOS; values are never clipped), lnZ is NaN there. */
int kpm_thermo(const double* d_mu, const double* d_ab, const kpm_problem* p, int32_t n,
               int32_t M, int32_t kernel, int32_t n_nodes, const double* d_T, int32_t n_T,
               double* d_lnZ, double* d_E, double* d_C, double* d_chi, uint8_t* d_znonpos,
               void* stream);

/* Thermodynamics in a magnetic field: the Zeeman term g mu_B B sum_i s^z_i of
 * the ladder Hamiltonian (Sec. III.A), H = H_0 + h S^z with h = g mu_B B in
 * energy units, at n_pts points (d_T[t], d_h[t]).  S^z commutes with H_0, so
 * every S^z > 0 sector enters twice, at m = +S^z and at its mirror m = -S^z,
 * with the zero-field DOS of the moments and energies E + h m; S^z = 0 once.
 * Outputs device [n_clusters][n_pts]: ln Z, E = <E> (Zeeman energy included),
 * C = (<E^2> - <E>^2)/T^2, chi = (<S_z^2> - <S_z>^2)/T, d_mag = <S_z> (may be
 * NULL; negative for h > 0), d_znonpos as in kpm_thermo.  Other arguments as
 * in kpm_thermo; at h = 0 the results equal kpm_thermo's up to rounding. */
int kpm_thermo_field(const double* d_mu, const double* d_ab, const kpm_problem* p, int32_t n,
                     int32_t M, int32_t kernel, int32_t n_nodes, const double* d_T,
                     const double* d_h, int32_t n_pts, double* d_lnZ, double* d_E, double* d_C,
                     double* d_chi, double* d_mag, uint8_t* d_znonpos, void* stream);

/* Workspace bytes for kpm_ftlm (0 if the arguments are invalid). */
size_t kpm_ftlm_workspace_size(const kpm_problem* p, int32_t n, const kpm_params* q);

/* Finite-temperature Lanczos method, the comparison method of the paper
 * (Introduction, Sec. III.C): for every start vector r of every problem (the
 * random vectors of chebyshev_moments: same kinds, seeds and streams, each
 * real column on its own), q->M steps of float64 Lanczos on the unscaled H
 * without reorthogonalisation (cut at the first off-diagonal below 1e-12 or
 * at the sector dimension) give Ritz values eps_j and squared first
 * eigenvector components; the estimator of Eq. (7) becomes
 *   Tr_Gamma f(H) ~ dim/R sum_r sum_j w_{rj} f(eps_{rj}),
 * with a complex vector's two real columns weighted by their share of |r|^2
 * (R = dim and weight 1 for the complete basis).  Thermodynamics as in
 * kpm_thermo_field at the points (d_T[t], d_h[t]) (d_h may be NULL: no field).
 *  q: M = Krylov dimension (>= 2), precision must be KPM_FP64; col_block
 *     batches columns into recursion blocks as for chebyshev_moments (each
 *     column keeps its own Lanczos coefficients); eps and the problems'
 *     bounds are not used
 *  outputs device [n_clusters][n_pts]: d_lnZ, d_E, d_C, d_chi, d_mag (<S_z>,
 *     may be NULL)
 *  d_ritz, d_weight: device double [columns][min(M, largest dim)] (may be
 *     NULL): Ritz values and estimator weights per real column (problem after
 *     problem), zero past each column's length
 * Errors: KPM_EINVAL, KPM_EWORKSPACE, KPM_EDEVICE (HIP error, or a tridiagonal
 * that did not converge). */
int kpm_ftlm(const kpm_problem* p, int32_t n, const kpm_params* q, const double* d_T,
             const double* d_h, int32_t n_pts, double* d_lnZ, double* d_E, double* d_C,
             double* d_chi, double* d_mag, double* d_ritz, double* d_weight, void* d_work,
             size_t work_bytes, void* stream);

/* Workspace bytes for kpm_sector_eigenvalues (0 if the arguments are invalid). */
size_t kpm_sector_eigenvalues_workspace_size(const kpm_problem* p, int32_t n, int32_t max_dim);

/* Exact spectra of the small sectors (Sec. II: a sector of small dimension is
 * diagonalised completely instead of being estimated stochastically).  For
 * every problem i whose sector dimension D (C(n_sites, n_up) for spin 1/2) is
 * <= max_dim, row i of d_evals gets the D eigenvalues of H (unscaled; the
 * problem's bounds are not used) on the sector, ascending, followed by NaN;
 * rows of larger sectors are all NaN.  Float64 throughout: the dense sector
 * matrix, Householder reduction to tridiagonal form (one column per step for
 * all sectors at once, spread over row tiles), every eigenvalue by bisection
 * on Sturm counts to the rounding level of the matrix.
 *  max_dim   1..1024
 *  d_evals   device double [n][max_dim]
 *  d_work    device workspace of kpm_sector_eigenvalues_workspace_size bytes
 *            (8 D^2 + 32 max(D, 4) per diagonalised sector + small tables), or
 *            NULL: allocated and freed inside the call
 * Errors: KPM_EINVAL, KPM_EWORKSPACE, KPM_EDEVICE (HIP error, or a neighbour
 * rank outside its sector). */
int kpm_sector_eigenvalues(const kpm_problem* p, int32_t n, int32_t max_dim, double* d_evals,
                           void* d_work, size_t work_bytes, void* stream);

/* Thermodynamics with exact small sectors: problem i with h_exact[i] != 0
 * (host uint8 [n]) contributes the C(n_sites, n_up) eigenvalues in row i of
 * d_evals (device double [n][evals_ld], as written by kpm_sector_eigenvalues),
 * each with the weight Ntil on which a dimension-D sector's DOS weights gamma_k
 * sum to Ntil * D; the other problems contribute their moments d_mu as in
 * kpm_thermo_field.  d_h may be NULL (no field).  Outputs as kpm_thermo_field.
 * Errors: KPM_EINVAL (also when an exact sector does not fit evals_ld),
 * KPM_ENOMEM, KPM_EDEVICE. */
int kpm_thermo_hybrid(const double* d_mu, const double* d_ab, const kpm_problem* p, int32_t n,
                      int32_t M, int32_t kernel, int32_t n_nodes, const double* d_evals,
                      int32_t evals_ld, const uint8_t* h_exact, const double* d_T, const double* d_h,
                      int32_t n_pts, double* d_lnZ, double* d_E, double* d_C, double* d_chi,
                      double* d_mag, uint8_t* d_znonpos, void* stream);

/* Derivative of L = sum_{c,T} wC[c][T] C[c][T] + wchi[c][T] chi[c][T] with
 * respect to the moments: d_lambda device double [n][M] = dL/dmu. */
int kpm_thermo_vjp(const double* d_mu, const double* d_ab, const kpm_problem* p, int32_t n,
                   int32_t M, int32_t kernel, int32_t n_nodes, const double* d_T, int32_t n_T,
                   const double* d_wC, const double* d_wchi, double* d_lambda, void* stream);

/* Workspace bytes for chebyshev_moments_vjp / kpm_thermo_grad. */
size_t chebyshev_moments_vjp_workspace_size(const kpm_problem* p, int32_t n,
                                            const kpm_params* q, int32_t ckpt_every);

/* Reverse-mode derivative of chebyshev_moments with the rescaling (a, b)
 * held fixed: given d_dmu = dL/dmu (device [n][M]) and the (a, b) used
 * forward (device [n][2]), writes d_dJ (device double, sum_p n_bonds(p)
 * entries, problem after problem in bond order) = dL/dJ_b.  The forward
 * recursion is recomputed from checkpoints taken every ckpt_every steps
 * (even, >= 2); with ckpt_every >= M/2 every vector of the forward pass is
 * kept (M/2 + 2 vectors in d_work) and nothing is recomputed.  The result
 * does not depend on ckpt_every.  Same seeds and vectors as
 * chebyshev_moments. */
int chebyshev_moments_vjp(const kpm_problem* p, int32_t n, const kpm_params* q,
                          const double* d_ab, const double* d_dmu, int32_t ckpt_every,
                          double* d_dJ, void* d_work, size_t work_bytes, void* stream);

/* The gradient in two calls, for callers that form dL/dmu themselves between
 * them (an autograd graph): chebyshev_moments_ckpt runs the recursion once,
 * writes the moments d_mu (device [n][M]) and the (a, b) it used d_ab (device
 * [n][2]; bounds as chebyshev_moments resolves them), and keeps the
 * recursion's checkpoints (every ckpt_every steps, even >= 2) in d_work;
 * chebyshev_moments_vjp_resume then runs only the reverse sweep of
 * chebyshev_moments_vjp from them.  d_work (caller-owned, both calls,
 * chebyshev_moments_ckpt_workspace_size bytes; NULL is refused) must hold
 * what the forward call left: the same p, n, q and ckpt_every, and no other
 * call on that memory in between.  Moments equal chebyshev_moments' to
 * rounding (the recursion may run on another kernel).
 * Errors: KPM_EINVAL, KPM_EWORKSPACE, KPM_EBOUNDS (forward), KPM_EDEVICE. */
size_t chebyshev_moments_ckpt_workspace_size(const kpm_problem* p, int32_t n, const kpm_params* q,
                                             int32_t ckpt_every);
int chebyshev_moments_ckpt(const kpm_problem* p, int32_t n, const kpm_params* q, int32_t ckpt_every,
                           double* d_mu, double* d_ab, void* d_work, size_t work_bytes, void* stream);
int chebyshev_moments_vjp_resume(const kpm_problem* p, int32_t n, const kpm_params* q,
                                 const double* d_ab, const double* d_dmu, int32_t ckpt_every,
                                 double* d_dJ, void* d_work, size_t work_bytes, void* stream);

/* Derivatives with respect to each cluster's couplings: the sectors of one
 * cluster (problems sharing its id) share its bond list, and Z is the sum over
 * sectors (Sec. II, below Eq. (9)), so dL/dJ_b of the cluster is the sum of
 * the per-sector derivatives.  d_dJ: device double, problem after problem in
 * bond order, as written by chebyshev_moments_vjp, chebyshev_moments_vjp_resume
 * or kpm_thermo_grad; d_dJ_cluster: device double, cluster after cluster (ids
 * ascending, 1 + largest id of them), each cluster's bonds in bond order (an
 * id with no problem contributes nothing).  Sums are formed in problem order
 * on `stream`, complete at return.  Errors: KPM_EINVAL (problems of one
 * cluster with different bond counts, invalid problems or NULL pointers),
 * KPM_ENOMEM, KPM_EDEVICE. */
int kpm_cluster_bond_grad(const kpm_problem* p, int32_t n, const double* d_dJ, double* d_dJ_cluster,
                          void* stream);

/* Loss and gradient in one call: moments, thermodynamics, their derivative
 * and the recursion adjoint, with the recursion run forward once (its
 * checkpointed pass gives the moments).  d_T [n_T], d_wC, d_wchi
 * [n_clusters][n_T]: device.  Outputs: d_L (device double [1]), d_dJ as in
 * chebyshev_moments_vjp, d_ab (device [n][2], may be NULL). */
int kpm_thermo_grad(const kpm_problem* p, int32_t n, const kpm_params* q, int32_t kernel,
                    int32_t n_nodes, const double* d_T, int32_t n_T, const double* d_wC,
                    const double* d_wchi, int32_t ckpt_every, double* d_L, double* d_dJ,
                    double* d_ab, void* d_work, size_t work_bytes, void* stream);

/* Debug export (host only): the site relabelling a block plan with L low
 * bits would use for spin-1/2 problem *p.  h_perm (host int32 [n_sites])
 * gets the new label of every site: labels 0..L-1 go to a set of L sites
 * that cuts few bonds (the first L sites unless a set with a strictly
 * smaller cut is found), the higher labels to the other sites in an order
 * where few bonds touch the highest labels (the slowest-varying bits of the
 * state words).  Returns 1 if relabelled, 0 if the identity is kept,
 * KPM_EINVAL for invalid arguments (spin s > 1/2, L outside 1..16). */
int kpm_site_relabel(const kpm_problem* p, int32_t L, int32_t* h_perm);

/* Launch statistics of the last chebyshev_moments call on this thread.
 * Host only (reads what the call recorded). */
typedef struct {
  int64_t step_launches;   /* recursion-step kernel launches (= M/2) */
  double bytes_per_launch; /* algorithmic HBM bytes of one step: 3 * storage
                              size * sum over blocks of dim * real columns,
                              + 4 * dim per block for the row and block
                              kernels (they stream the 4-byte state words);
                              the block-table kernel reads per-block tables
                              instead: per block of low-bit states
                              12 + 6 * (high-high bonds) + 4 * (mixed bonds);
                              the spin-s kernel reads 8 + 8 * n_bonds per row
                              (digit string, neighbour-rank slots) */
  double state_col_steps;  /* sum over blocks of dim * real columns * steps */
  int32_t col_block;       /* real columns per block chosen */
  int32_t rows_per_tile;   /* basis states per workgroup tile (block kernels: mean) */
  int32_t graph_segment;   /* steps per captured graph (0 = direct launches) */
  int32_t kernel;          /* step kernel used: 0 column-chunk, 1 row, 2 block,
                              3 block-table, 4 spin-s, 5 slice (block-table
                              tiles, each wave on rows of one block) */
  double recursion_ms;     /* hipEvent time on the call's stream from the first
                              to the last recursion-step launch, inclusive */
  int32_t relabelled;      /* problems whose sites the block kernels relabel (fewer
                              bonds between the low and the high bits; results are
                              unchanged: start vectors and exported rows keep the
                              original basis order) */
  int32_t waves;           /* waves per workgroup of the step kernel (slice
                              kernel: 1, or 2 / 4 sharing one tile; others 1) */
} kpm_run_stats;
int kpm_last_run_stats(kpm_run_stats* out);

/* Forget every autotuned launch shape (the next autotuned call measures again). */
int kpm_autotune_reset(void);

#ifdef __cplusplus
}
#endif
#endif /* KPM_H */

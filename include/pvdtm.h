/*
 * pvdtm.h -- C ABI of the MI355X (gfx950) matrix-free Chebyshev/stencil library.
 *
 * Operations follow Pieper, Hager, Fehske, "A domain-specific language and
 * matrix-free stencil code for investigating electronic properties of Dirac
 * and topological materials" (arXiv:1708.09689):
 *   - lattice + stencil description: Sec. 3.2 (stencil blocks per neighbour
 *     offset), Sec. 3.4 (cuboid geometry, per-dimension periodic BCs);
 *   - model stencils: Sec. 2.1 (graphene), 2.2 (3D TI), 2.3 (Weyl);
 *   - fused sweep y = alpha (H - beta) x + gamma y with partial dot products:
 *     Sec. 3.2, generated-code listing (scale_h, shift_h, scale_z, dot_xx/xy/yy);
 *   - start vectors: Sec. 3.4 (initial-vector callback), Sec. 3.3 and 4.2
 *     (random blocks from the counter-based generator, for the stochastic
 *     trace);
 *   - KPM moments: Sec. 2.2 (DOS) and Sec. 4;
 *   - Chebyshev time propagation: Sec. 4.1, Eq. (U_1);
 *   - Chebyshev filter diagonalisation with Rayleigh-Ritz: Sec. 4.2.
 *
 * Conventions
 * -----------
 * Data layout.  A block of nb vectors is stored row-major [rows][nb], complex
 * interleaved (re, im).  Row r = s*n_orb + o, site s = x + Lx*(y + Ly*z);
 * element (x, y, z, o, c) is complex number ((s*n_orb + o)*nb + c).  x is the
 * fastest lattice direction.
 * Device pointers.  Every vector, potential, moment or gradient pointer is a
 * device pointer (hipMalloc'd, or a torch CUDA tensor's data_ptr()); it is
 * BORROWED: the caller keeps it alive until the work queued on `stream` has
 * finished.  Complex128 blocks must be 16-byte aligned, complex64 8-byte.
 * Host pointers.  Descriptors, coefficient arrays and scale/shift arrays are
 * host memory, copied or consumed before the call returns.
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = default stream).
 * All launches are asynchronous on that stream unless a function says it
 * synchronises.
 * Errors.  Every argument is validated before the first launch; on error
 * nothing is queued, the status is returned and pv_last_error() (thread
 * local) holds a message.  No C++ exception crosses this interface.
 * PV_ERR_OOM: the lattice's device tables (made on its first use on a
 * device) could not be allocated; the lattice stays usable and the next
 * call tries again.  For tests, the environment variable
 * PV_TEST_FAIL_DEVICE_ALLOC forces the failure: "all", or k to fail only
 * the k-th allocation of a set-up (1 coefficients, 2 generic stencil
 * offsets, 3 the zero row).
 * PV_ERR_NONFINITE: results read on the host hold NaN or Inf -- moments
 * passed to pv_kpm_dos / pv_kpm_spectral_function, or the Gram and Lanczos
 * matrices of pv_chebfd and pv_trlanczos_fd (a non-finite start block or
 * field); the outputs are then not written.
 * Workspace.  Functions that need scratch device memory take (work,
 * work_bytes) from the caller; the matching *_workspace_size() call gives the
 * minimum size.  Too small a workspace gives PV_ERR_WORKSPACE.
 * Determinism.  Reductions use fixed-order two-pass sums (no floating-point
 * atomics): repeated calls with the same inputs give bitwise equal results.
 * Threads.  Calls from several host threads may run at once on different
 * objects, or on one lattice or batch when none of them changes it
 * (set_potential, set_random_potential, set_tuning, autotune and the batch
 * calls, which rebuild their graph, change it); the caller serialises
 * changes of an object against every other use of it.
 */
#ifndef PVDTM_H
#define PVDTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pv_status {
    PV_OK = 0,
    PV_ERR_INVALID_ARG = 1,
    PV_ERR_UNSUPPORTED = 2,
    PV_ERR_NOT_HERMITIAN = 3,
    PV_ERR_WORKSPACE = 4,
    PV_ERR_OOM = 5,
    PV_ERR_HIP = 6,
    PV_ERR_NONFINITE = 7,
    PV_ERR_NO_DEVICE = 8,
    PV_ERR_NOT_CONVERGED = 9
} pv_status;

/* Vector element type: complex128 or complex64 (FP32 vectors, FP64 dots). */
typedef enum pv_dtype { PV_C128 = 0, PV_C64 = 1 } pv_dtype;
/* Real type of the on-site field array. */
typedef enum pv_rtype { PV_F64 = 0, PV_F32 = 1 } pv_rtype;
/* How the real on-site field V enters H (Sec. 2): */
typedef enum pv_pot_mode {
    PV_POT_NONE = 0,     /* no field */
    PV_POT_SITE = 1,     /* V[s] times the identity on the site's orbitals (V_n Gamma^0) */
    PV_POT_ORBITAL = 2   /* V[s*n_orb + o] on the diagonal (v_{n,j} of the graphene cell) */
} pv_pot_mode;

#define PV_CHECK_HERMITIAN 1u

/* Partial dot products requested from a sweep (Sec. 3.2 listing flags). */
#define PV_DOT_XX 1u  /* <x, x>          */
#define PV_DOT_XY 2u  /* <x, y_new>      */
#define PV_DOT_YY 4u  /* <y_new, y_new>  */

#define PV_MAX_TERMS 26
#define PV_MAX_ORB 4
#define PV_MAX_NB 64

/*
 * Lattice and stencil (Sec. 3.2, Sec. 3.4).  The operator is
 *     (H x)[s] = sum_t B_t x[s + d_t] + (E0 + V_s) x[s]
 * with d_t in {-1,0,1}^3 \ {0}; a neighbour that leaves [0, L) along an open
 * dimension contributes nothing, along a periodic one it wraps.
 *   dim       2 or 3 (dim 2 requires L[2] == 1 and d_t[2] == 0)
 *   L         extents (x, y, z), each >= 1
 *   n_orb     orbitals per site: 1, 2 or 4
 *   periodic  per-dimension flag (nonzero = periodic)
 *   n_terms   number of neighbour offsets, 0..PV_MAX_TERMS, pairwise distinct
 *   offsets   [n_terms][3]
 *   blocks    [n_terms][n_orb][n_orb] complex as (re, im) doubles; block[t][o][o']
 *             multiplies x[s + d_t, o'] into row o
 *   onsite    [n_orb][n_orb] complex (E0)
 *   pot_mode  pv_pot_mode
 *   flags     PV_CHECK_HERMITIAN: require B_{-d} = B_d^H and E0 = E0^H
 *             (to 1e-14 relative); otherwise PV_ERR_NOT_HERMITIAN
 */
typedef struct pv_lattice_desc {
    int dim;
    int64_t L[3];
    int n_orb;
    int periodic[3];
    int n_terms;
    const int *offsets;
    const double *blocks;
    const double *onsite;
    int pot_mode;
    unsigned flags;
} pv_lattice_desc;

typedef struct pv_lattice pv_lattice;
typedef struct pv_batch pv_batch;

/* Thread-local message describing the last error of this thread. */
const char *pv_last_error(void);
const char *pv_status_string(pv_status s);
int pv_version(void);
/* Hash of the sources and this header the library was built from (16 hex
 * digits, "unstamped" for builds that did not set it).  A binding compares it
 * with the sources it was shipped with, so that structures such as
 * pv_tuning never cross the interface with two different layouts. */
const char *pv_source_hash(void);

/*
 * Model stencils (host only, no device use).  Fill the descriptor arrays for
 * a model of Sec. 2; the caller provides capacity offsets[PV_MAX_TERMS*3],
 * blocks[PV_MAX_TERMS*PV_MAX_ORB*PV_MAX_ORB*2], onsite[PV_MAX_ORB*PV_MAX_ORB*2].
 *   PV_MODEL_TI         Sec. 2.2 Eq. (TB_H_topi); params {t, m, Delta1, Delta2};
 *                       Gamma^1 = tau_z sigma_0, Gamma^{j+1} = tau_x sigma_j,
 *                       Gamma^5 = tau_y sigma_0, orbital o = 2 tau + sigma;
 *                       hopping -(t/2)(G1 - i G_{j+1}) from n to n + e_j
 *   PV_MODEL_GRAPHENE2  honeycomb, two-site cell on an (i, j) grid; params {t}:
 *                       A(i,j) bonds to B(i,j), B(i-1,j), B(i,j-1) with -t
 *   PV_MODEL_GRAPHENE4  Sec. 2.1 Eq. (graphene_model) four-site cell; params {t}
 *   PV_MODEL_WEYL       Sec. 2.3 Eq. (TB_H_wsm); params {k0}
 * On return *n_terms, *n_orb, *dim and *pot_mode describe the model.
 */
/*
 * Stencil description language (Sec. 3.2): parse the text of a DSL program
 * into the same descriptor arrays as pv_model_stencil (same capacities).
 * Statements: dim, size, n_coeff_const, n_coeff_variable, n_coeff_rand,
 * coeff_const_default, and "nn d0 d1 [d2]" followed by one row line per
 * orbital with entries "col|value" or "col|type|arg" (type f fixed, c
 * constant coefficient, v variable per site, r random per site).  Entry
 * (k, q) of the block at offset d adds value * x[s + d][q] to y[s][k].
 * Values may be complex ("0.5i", "1-2i"; an extension of the paper's real
 * coefficients).  Constant coefficients take coeff_const[idx] when idx <
 * n_const, else the coeff_const_default values.  Per-site coefficients are
 * accepted on the on-site diagonal only: *pot_mode = PV_POT_SITE (one index
 * for all orbitals) or PV_POT_ORBITAL (index k on row k), and *field_kind =
 * 1 for v (attach an array with pv_lattice_set_potential) or 2 for r (use
 * pv_lattice_set_random_potential); 0 without per-site coefficients.
 * Syntax errors return PV_ERR_INVALID_ARG with the line number in
 * pv_last_error(); shapes the kernels do not support, PV_ERR_UNSUPPORTED.
 */
pv_status pv_dsl_stencil(const char *text, const double *coeff_const, int n_const, int *dim,
                         int *n_orb, int *n_terms, int *offsets, double *blocks, double *onsite,
                         int *pot_mode, int *field_kind);

typedef enum pv_model {
    PV_MODEL_TI = 0, PV_MODEL_GRAPHENE2 = 1, PV_MODEL_GRAPHENE4 = 2, PV_MODEL_WEYL = 3
} pv_model;
pv_status pv_model_stencil(int model, const double *params, int *dim, int *n_orb,
                           int *n_terms, int *offsets, double *blocks, double *onsite,
                           int *pot_mode);

/* Create a lattice from a descriptor (host only; the library copies it and
 * owns *out).  pv_lattice_destroy frees library state only. */
pv_status pv_lattice_create(const pv_lattice_desc *desc, pv_lattice **out);
void pv_lattice_destroy(pv_lattice *lat);

/* Number of sites, rows (sites * n_orb) and the sweep kernel family chosen
 * for this stencil (0 = generic dense blocks, >0 = a pattern-specialised
 * kernel whose zero / real / imaginary block structure is compiled in). */
pv_status pv_lattice_info(const pv_lattice *lat, int64_t *n_sites, int64_t *n_rows,
                          int *kernel_family);

/* Attach the on-site field: V_dev is a BORROWED device array of n_sites
 * (PV_POT_SITE) or n_rows (PV_POT_ORBITAL) reals of type rtype; NULL means
 * V = 0.  Replaces any previous field. */
pv_status pv_lattice_set_potential(pv_lattice *lat, const void *V_dev, int rtype);

/*
 * On-the-fly disorder (Sec. 3.3: random numbers generated inside the kernel
 * instead of streamed from memory).  The field is never stored: the sweep
 * kernels evaluate it wherever they need it from a counter-based generator,
 *     V[i] = W * (u_i - 1/2),  u_i = (s_i >> 11) * 2^-53,
 *     s_i  = output number i + 1 of SplitMix64 (Steele, Lea, Flood 2014)
 *            seeded with `seed`,
 * i the site index (PV_POT_SITE) or the orbital row (PV_POT_ORBITAL).  The
 * value is the same in every sweep and independent of the traversal order;
 * it saves the field's 8 / (n_orb nb) bytes per row update.  Replaces any
 * previous field (pv_lattice_set_potential replaces this one in turn).
 * Gradients with respect to the field are still returned per site / row.
 */
pv_status pv_lattice_set_random_potential(pv_lattice *lat, uint64_t seed, double W);

/*
 * One fused sweep (Sec. 3.2 listing), per column c of the nb-wide blocks:
 *     y[:, c] = alpha[c] * (H x[:, c] - beta[c] x[:, c]) + gamma[c] * z[:, c]
 * gamma[c] == 0 means z is not read (z may be NULL then for all columns).
 * z may equal y (in-place recurrence); x must not overlap y or z.
 * alpha, beta, gamma: host arrays [nb].  dot_flags selects partial dot
 * products written to dots (device, [nb][4] doubles: <x,x>, Re<x,y>,
 * Im<x,y>, <y,y>, accumulated in FP64); dots may be NULL when dot_flags==0.
 * nb: power of two, 1..PV_MAX_NB.  Workspace: pv_spmmv_workspace_size().
 */
size_t pv_spmmv_workspace_size(const pv_lattice *lat, int dtype, int nb);
pv_status pv_spmmv(pv_lattice *lat, int dtype, int nb, const void *x, const void *z, void *y,
                   const double *alpha, const double *beta, const double *gamma,
                   unsigned dot_flags, double *dots, void *work, size_t work_bytes,
                   void *stream);

/*
 * pv_spmmv without allocation, for callers that cannot call hipMalloc: code
 * under HIP graph capture, tight serving loops, harnesses that forbid device
 * allocation.  Same arguments, semantics and errors as pv_spmmv, without
 * (work, work_bytes): the partial dot products and the per-column scale
 * table live in a library-owned static device array of
 * PV_NOALLOC_SCRATCH_BYTES, one copy per GPU, held until the process ends.
 * No call allocates or frees device memory.
 *   - PV_ERR_UNSUPPORTED when pv_spmmv_workspace_size(lat, dtype, nb)
 *     exceeds PV_NOALLOC_SCRATCH_BYTES.
 *   - PV_ERR_INVALID_ARG when the lattice has no device tables on the current
 *     device yet: the first other sweep call there (pv_spmmv, pv_kpm_moments,
 *     ...) creates them.
 *   - Every call on one GPU shares that GPU's array and leaves its contents
 *     behind; calls that overlap on one GPU (several streams or host threads)
 *     race, so the caller serialises them.  Per-column (non-uniform) alpha,
 *     beta, gamma synchronise the stream, as in pv_spmmv.
 *   - Generic stencils (generated kernels, see pv_lattice_set_codegen) take
 *     a generated kernel only when an earlier call on this GPU loaded that
 *     instance, else the interpreted generic kernel: compiling and loading
 *     one allocates.
 */
#define PV_NOALLOC_SCRATCH_BYTES (64 << 20)
pv_status pv_spmmv_noalloc(pv_lattice *lat, int dtype, int nb, const void *x, const void *z, void *y,
                           const double *alpha, const double *beta, const double *gamma, unsigned dot_flags,
                           double *dots, void *stream);

/*
 * Vector block from a host callback (Sec. 3.4: the initial-vector interface
 * of the paper's library).  For every site (x, y, z), orbital o and column k,
 * with r = {x, y, z, o}:
 *     Re out[(s*n_orb + o)*nb + k] = fnc(r, k, parm, seed)
 *     Im out[...]                  = fnc_im(r, k, parm, seed)  (0 if NULL)
 * called on the host by one thread in memory order (column fastest, then
 * orbital, x, y, z).  parm is handed through; seed points to a 128-bit state (two uint64_t) that the
 * library sets from `seed_value` (SplitMix64 outputs 1 and 2 of the stream
 * seeded with it) before the first call, for the callback's own random
 * draws.  out: device block of dtype (complex64 takes the values rounded to
 * FP32), n_rows x nb, written by a copy queued on `stream` after its earlier
 * work; the call returns when out holds the block.  Host memory for one block is allocated for the copy
 * (PV_ERR_OOM if it cannot be).
 */
typedef double (*pv_vector_func)(const int64_t *r, int k, void *parm, void *seed);
pv_status pv_vector_from_func(pv_lattice *lat, int dtype, int nb, pv_vector_func fnc, pv_vector_func fnc_im,
                              void *parm, uint64_t seed_value, void *out, void *stream);

/*
 * Random start blocks for the stochastic trace of KPM (Sec. 4.2), generated
 * on the device.  Sec. 3.4 fills vectors from a function of the site, the
 * orbital, the column and a random seed; here every entry is a pure function
 * of (seed, global element index), from the counter-based generator of the
 * on-the-fly field (SplitMix64, Sec. 3.3): element (r, c) of out takes index
 * i = (row0 + r) * nb + c and z_i = output number i + 1 of the stream seeded
 * with seed, and
 *     kind PV_RANDOM_PHASE:  exp(i phi), phi = 2 pi u, u = (z_i >> 11) 2^-53
 *                            (cos and sin in FP64)
 *     kind PV_RANDOM_Z4:     i^k, k = z_i >> 62: 1, i, -1 or -i
 * PV_C64 blocks hold the FP64 values rounded to FP32.  out: device block of
 * dtype, n_rows x nb (rows row0 .. row0 + n_rows - 1 of a block over a larger
 * row range; row0 = 0 for the lattice's own block), written.  row0 >= 0 and
 * (row0 + n_rows) * nb < 2^63, else PV_ERR_INVALID_ARG before any launch.
 */
#define PV_RANDOM_PHASE 0
#define PV_RANDOM_Z4 1
pv_status pv_random_block(pv_lattice *lat, int dtype, int nb, uint64_t seed, int kind, int64_t row0, void *out,
                          void *stream);

/*
 * KPM moments (Sec. 2.2 DOS, Sec. 4): for every column c of the start block r
 *     mu[c][n] = Re <r_c, T_n(H~) r_c> / D,  H~ = (H - b)/a,  n = 0..M-1,
 * with D = n_rows, formed from M/2 fused sweeps through
 * mu_{2n} = 2<w_n,w_n>/D - mu_0 and mu_{2n+1} = 2 Re<w_n,w_{n+1}>/D - mu_1.
 * M even, 2 <= M <= 65536; a > 0.  r is read only.  mu: device [nb][M] FP64.
 */
size_t pv_kpm_workspace_size(const pv_lattice *lat, int dtype, int nb, int M);
pv_status pv_kpm_moments(pv_lattice *lat, int dtype, int nb, int M, double a, double b,
                         const void *r, double *mu, void *work, size_t work_bytes, void *stream);

/* Jackson-damped DOS per row from moments (host arrays):
 *   rho(E) = [g_0 mu_0 + 2 sum_{n>=1} g_n mu_n T_n(x)] / (pi a sqrt(1 - x^2)),
 *   x = (E - b)/a; mu: [M] (e.g. the column mean), E, rho: [nE]. */
pv_status pv_kpm_dos(int M, const double *mu, double a, double b, int nE, const double *E,
                     double *rho);

/*
 * Momentum-resolved spectral function (Sec. 2.2, Eq. ak) by KPM with Bloch
 * start columns.  pv_bloch_block writes the block
 *     out[s][o][c] = exp(i k_c . r_s)  if o == orbital[c] and r_s lies in
 *                                      the layer, else 0,
 * r_s = (x, y, z) the site's integer coordinates, k: host [nb][3] (radians
 * per lattice unit), orbital: host [nb] in [0, n_orb).  layer_axis = -1 puts
 * the state on every site; 0, 1 or 2 restricts it to the sites whose
 * coordinate along that axis equals layer_index (a test state on one
 * surface, as for the Fermi arcs of Sec. 4.3).  out: device block of dtype,
 * n_rows x nb.  With mu = pv_kpm_moments of that block,
 * pv_kpm_spectral_function returns on the host
 *     A(E) = norm * sum_c rho_c(E),
 * rho_c the Jackson-damped reconstruction of column c (as pv_kpm_dos).
 * norm = n_rows / (number of sites carrying the state) makes A integrate to
 * the number of columns: the spectral weight per site of Eq. ak.
 */
pv_status pv_bloch_block(pv_lattice *lat, int dtype, int nb, const double *k, const int *orbital,
                         int layer_axis, int64_t layer_index, void *out, void *stream);
pv_status pv_kpm_spectral_function(int nb, int M, const double *mu, double a, double b, double norm,
                                   int nE, const double *E, double *A);

/*
 * Chebyshev series applied to a block (Sec. 4.1 and 4.2):
 *     Y = sum_{k=0}^{K} coef[k] T_k(H~) X,   coef: host complex [K+1] (re, im)
 * using K fused sweeps whose epilogue accumulates coef[k] * w_k.  X and Y
 * must not overlap.  K >= 0.
 */
size_t pv_cheb_series_workspace_size(const pv_lattice *lat, int dtype, int nb);
pv_status pv_cheb_series(pv_lattice *lat, int dtype, int nb, double a, double b, int K,
                         const double *coef, const void *X, void *Y, void *work,
                         size_t work_bytes, void *stream);

/*
 * Chebyshev time propagation, Sec. 4.1 Eq. (U_1): nsteps steps of
 *     psi <- exp(-i b dt) [c_0 + 2 sum_{k=1}^{M} c_k T_k(H~)] psi,
 *     c_k = (-i)^k J_k(a dt)   (Bessel J_k by Miller's backward recurrence)
 * in place on psi (device [rows][nb]).  M >= 1, nsteps >= 0.
 */
size_t pv_cheb_propagate_workspace_size(const pv_lattice *lat, int dtype, int nb);
pv_status pv_cheb_propagate(pv_lattice *lat, int dtype, int nb, double a, double b, double dt,
                            int M, int nsteps, void *psi, void *work, size_t work_bytes,
                            void *stream);
/* c_k = (-i)^k J_k(a dt), k = 0..M, complex (re, im) into host coef[M+1][2]. */
pv_status pv_cheb_tp_coefficients(double a, double dt, int M, double *coef);

/*
 * Tall-skinny products with FP64 accumulation (Rayleigh-Ritz of Sec. 4.2):
 *   pv_gram:         G[i][j] = sum_r conj(X[r][i]) Y[r][j]
 *                    X [rows][nx], Y [rows][ny], G device complex128 [nx][ny]
 *   pv_block_rotate: Y[r][j] = (accumulate ? Y[r][j] : 0) + sum_i X[r][i] Q[i][j]
 *                    X [rows][nx], Q device complex128 [nx][ny], Y [rows][ny]
 *                    (Y must not overlap X); sums in FP64
 * nx, ny in 1..PV_MAX_NB.
 */
size_t pv_gram_workspace_size(int64_t rows, int nx, int ny);
pv_status pv_gram(int dtype, int64_t rows, int nx, int ny, const void *X, const void *Y,
                  double *G, void *work, size_t work_bytes, void *stream);
pv_status pv_block_rotate(int dtype, int64_t rows, int nx, int ny, const void *X,
                          const double *Q, int accumulate, void *Y, void *stream);

/*
 * Chebyshev filter diagonalisation, Sec. 4.2: interior eigenpairs of H in the
 * window [lam_l, lam_r] (energy units, inside [b - a, b + a]).  Each
 * iteration filters the search space X (ns = bw * nblk columns, stored as
 * nblk device blocks [rows][bw] back to back, i.e. [nblk][rows][bw]) with
 *     p(H~) = sum_{k=0}^{degree} g_k c_k T_k(H~),
 *     c_0 = (acos x_l - acos x_r)/pi, c_k = 2 (sin(k acos x_l) - sin(k acos x_r))/(k pi),
 *     g_k Jackson damping, x = (lam - b)/a,
 * orthonormalises it with Cholesky QR applied twice (FP64 Gram and host
 * factorisation), and performs Rayleigh-Ritz: H_S = Q^H H Q (FP64), host
 * Jacobi eigensolver, X <- Q U with Ritz pairs ordered by |theta - centre|,
 * residuals ||H x_i - theta_i x_i|| from a shifted sweep with fused <y,y>.
 * A pair has converged when theta lies in the window and its residual is
 * <= tol (Ritz values of a search space larger than the window's count that
 * belong to no eigenvector keep large residuals and never count).  Stops
 * when n_target pairs have converged, or after max_iter iterations
 * (PV_ERR_NOT_CONVERGED; outputs still filled).  Synchronises the stream.
 * In/out: X (start block -> Ritz vectors, converged ones first, each group
 * ordered by |theta - centre|); out: theta[ns], res[ns] (host, same order),
 * *n_conv (converged pairs among the first n_target), *iters.  The Gram
 * matrices and rotations of the whole search space run as one pass each.
 */
size_t pv_chebfd_workspace_size(const pv_lattice *lat, int dtype, int bw, int nblk);
pv_status pv_chebfd(pv_lattice *lat, int dtype, int bw, int nblk, double a, double b,
                    double lam_l, double lam_r, int degree, int n_target, double tol,
                    int max_iter, void *X, double *theta, double *res, int *n_conv, int *iters,
                    void *work, size_t work_bytes, void *stream);
/* g_k c_k, k = 0..K, of the ChebFD window filter (host). */
pv_status pv_chebfd_filter_coefficients(double lam_l, double lam_r, double a, double b, int K,
                                        double *coef);
/* Host Hermitian eigensolver used by Rayleigh-Ritz (cyclic Jacobi, FP64):
 * A complex row-major [n][n] (re, im), w ascending [n], V [n][n] complex with
 * the eigenvectors as columns. */
pv_status pv_host_heev(int n, const double *A, double *w, double *V);

/*
 * trLanczosFD (Sec. 4.2, Tab. fd_cases): thick-restart block Lanczos with
 * polynomial filtering (Li, Xi, Vecharynski, Yang, Saad, SIAM J. Sci.
 * Comput. 2016) for the eigenpairs of H inside [lam_l, lam_r].
 *   filter  p(x) = sum_k g_k (2 - delta_k0) T_k(x_c) T_k(x) / norm, the
 *           Jackson-damped delta peak at the window centre x_c (scaled units
 *           x = (E - b)/a), p(x_c) = 1; tau = min(p(x_l), p(x_r)).
 *           pv_trlanczos_filter returns coef[K+1] and tau (host only).
 *   solver  block Lanczos on p(H~) with blocks of nbl columns (each step =
 *           one Chebyshev series of degree `degree` on nbl columns; nbl >= 2
 *           resolves the Kramers pairs of the TI), full reorthogonalisation
 *           (FP64 Gram, twice), Cholesky QR (twice) of every new block, a
 *           basis of m vectors; after m vectors the Ritz vectors of p(H~)
 *           with values above tau, rounded up to whole blocks, are kept
 *           (thick restart).  Converged when every kept pair above tau has
 *           ||H u - theta u|| <= tol and their number did not change since
 *           the previous restart; the pairs returned are those with theta
 *           inside the window.
 * v0: device start block [n_rows][nbl] (not modified).  Outputs (host):
 * theta and res [m] (the first *n_found entries, theta ascending),
 * *restarts; the first min(*n_found, n_out) Ritz vectors into X
 * [n_rows][n_out] (n_out a power of two <= PV_MAX_NB, or 0 with X NULL).
 * PV_ERR_NOT_CONVERGED after max_restarts with the current pairs returned.
 * nbl a power of two <= 32, m a multiple of nbl, 2 nbl <= m, m + nbl <= 1024.
 */
pv_status pv_trlanczos_filter(double lam_l, double lam_r, double a, double b, int K, double *coef,
                              double *tau);
size_t pv_trlanczos_workspace_size(const pv_lattice *lat, int dtype, int nbl, int m);
pv_status pv_trlanczos_fd(pv_lattice *lat, int dtype, double a, double b, double lam_l, double lam_r,
                          int degree, int nbl, int m, double tol, int max_restarts, const void *v0,
                          int n_out, void *X, double *theta, double *res, int *n_found, int *restarts,
                          void *work, size_t work_bytes, void *stream);

/*
 * Gradients with respect to the on-site field V (discrete adjoints of the
 * recurrences above; a and b are fixed numbers, not differentiated).
 *
 * pv_kpm_moments_vjp: for L = sum_{c,n} gbar[c][n] mu[c][n] (mu as computed
 * by pv_kpm_moments), gradV = dL/dV.  With N = M/2 and w_k = T_k(H~) r, the
 * adjoint vectors follow lambda_k = G_k + 2 H~ lambda_{k+1} - lambda_{k+2}
 * (k = N..1), G_k = dL/dw_k from the product doubling, and
 *   dL/dV_m = (1/a) Re [<lambda_1, P_m w_0> + 2 sum_{k=1}^{N-1} <lambda_{k+1}, P_m w_k>]
 * (P_m: rows of site m, or row m for PV_POT_ORBITAL).  The forward vectors are
 * checkpointed in pairs every ckpt_every steps and recomputed per segment.
 * gbar: device [nb][M]; gradV: device [n_sites] (site field) or [n_rows]
 * (orbital field), overwritten.  Needs n_orb*nb <= 64 for a site field.
 * Asynchronous on the stream: gbar is read on the device (a kernel turns it
 * into the coefficients of the G_k), so it may be produced by earlier work
 * on the same stream.
 *
 * pv_cheb_propagate_vjp: for psi_T = U(dt)^nsteps psi0 (pv_cheb_propagate)
 * and a cotangent psibar (dL = Re <psibar, d psi_T>), returns gradV = dL/dV
 * and, if psi0bar != NULL, the cotangent of psi0.  Every step is reversed
 * with the Clenshaw-type adjoint of the series sum_k eta_k T_k(H~).
 */
size_t pv_kpm_vjp_workspace_size(const pv_lattice *lat, int dtype, int nb, int M, int ckpt_every);
pv_status pv_kpm_moments_vjp(pv_lattice *lat, int dtype, int nb, int M, double a, double b,
                             const void *r, const double *gbar, double *gradV, int ckpt_every,
                             void *work, size_t work_bytes, void *stream);

/*
 * The same gradient split in two calls for a caller that needs the moments
 * before the cotangent is known (reverse-mode autodiff):
 * pv_kpm_moments_ckpt computes mu exactly as pv_kpm_moments does and writes
 * the checkpoint pairs (w_{jC}, w_{jC+1}) into `work` as it goes (sized by
 * pv_kpm_vjp_workspace_size, with the same ckpt_every);
 * pv_kpm_moments_vjp_ckpt then runs only the segment recomputation and the
 * adjoint sweep of pv_kpm_moments_vjp from that workspace.  The caller keeps
 * `work`, r and the field unchanged between the two calls and passes the
 * same lat, dtype, nb, M, a, b, r and ckpt_every to both; the result equals
 * pv_kpm_moments_vjp's, and the second call may be repeated (other
 * cotangents) on the same workspace.  With ckpt_every >= M/2 the forward
 * keeps every w_k (M/2 + 6 vectors of workspace) and the adjoint recomputes
 * none.  Both calls are asynchronous on the stream.
 */
pv_status pv_kpm_moments_ckpt(pv_lattice *lat, int dtype, int nb, int M, double a, double b,
                              const void *r, double *mu, int ckpt_every, void *work,
                              size_t work_bytes, void *stream);
pv_status pv_kpm_moments_vjp_ckpt(pv_lattice *lat, int dtype, int nb, int M, double a, double b,
                                  const void *r, const double *gbar, double *gradV, int ckpt_every,
                                  void *work, size_t work_bytes, void *stream);
size_t pv_cheb_propagate_vjp_workspace_size(const pv_lattice *lat, int dtype, int nb, int M,
                                            int nsteps);
pv_status pv_cheb_propagate_vjp(pv_lattice *lat, int dtype, int nb, double a, double b, double dt,
                                int M, int nsteps, const void *psi0, const void *psibar,
                                void *psi0bar, double *gradV, void *work, size_t work_bytes,
                                void *stream);

/*
 * The propagation gradient split in two calls, for reverse-mode autodiff:
 * pv_cheb_propagate_keep writes psiT = U(dt)^nsteps psi0 (psiT must not
 * alias psi0; psi0 is not modified) and keeps psi_1..psi_{nsteps-1} in
 * `work`; with keep_series != 0 it also keeps every step's Chebyshev
 * vectors w_1..w_M (nsteps*M more vectors), so that the adjoint recomputes
 * none.  `work` is sized by pv_cheb_propagate_keep_workspace_size (with
 * keep_series = 0 it equals pv_cheb_propagate_vjp_workspace_size).
 * pv_cheb_propagate_vjp_keep then runs only the reverse steps of
 * pv_cheb_propagate_vjp from what was kept.  The caller keeps `work`, psi0
 * and the field unchanged between the calls and passes the same arguments
 * (keep_series included) to both; the second call may be repeated (other
 * cotangents).  Results equal pv_cheb_propagate's and
 * pv_cheb_propagate_vjp's up to rounding.
 */
size_t pv_cheb_propagate_keep_workspace_size(const pv_lattice *lat, int dtype, int nb, int M,
                                             int nsteps, int keep_series);
pv_status pv_cheb_propagate_keep(pv_lattice *lat, int dtype, int nb, double a, double b, double dt,
                                 int M, int nsteps, const void *psi0, void *psiT, int keep_series,
                                 void *work, size_t work_bytes, void *stream);
pv_status pv_cheb_propagate_vjp_keep(pv_lattice *lat, int dtype, int nb, double a, double b,
                                     double dt, int M, int nsteps, const void *psi0,
                                     const void *psibar, void *psi0bar, double *gradV,
                                     int keep_series, void *work, size_t work_bytes, void *stream);

/*
 * Batched KPM over independent lattices (disorder realisations, possibly of
 * different sizes) of one stencil family: every Chebyshev step of all
 * instances is ONE kernel launch (each workgroup serves one instance, argument
 * records in a device table) followed by one per-instance fixed-order
 * reduction; the M/2 steps are captured into a HIP graph on the first call and
 * replayed on later calls with identical arguments (r pointers, a, b, fields,
 * workspace); the graph writes the moments into the workspace and each call
 * then copies them to mu, so mu may differ between calls.  Per instance i: mu[i][c][n] = Re <r_i,c, T_n(H~_i) r_i,c> / D_i,
 * H~_i = (H_i - b[i]) / a[i].  r: host array of n device pointers; mu: device
 * [n][nb][M].  The library owns the lattice list (borrowed lattices must
 * outlive the batch) and the graph; the workspace holds the argument tables,
 * so it must stay allocated while the graph may be replayed.
 */
pv_status pv_batch_create(int n, pv_lattice *const *lats, pv_batch **out);
void pv_batch_destroy(pv_batch *batch);
size_t pv_batch_kpm_workspace_size(const pv_batch *batch, int dtype, int nb, int M);
pv_status pv_batch_kpm_moments(pv_batch *batch, int dtype, int nb, int M, const double *a,
                               const double *b, const void *const *r, double *mu, void *work,
                               size_t work_bytes, void *stream);
/* Number of graph captures and replays performed so far (diagnostics). */
pv_status pv_batch_stats(const pv_batch *batch, int *captures, int *replays);

/* Scalar helper used to measure achievable bandwidth: dst = src (bytes, a
 * multiple of 16), a plain streaming copy kernel. */
pv_status pv_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Second bandwidth reference with the stream mix of one Chebyshev step (two
 * reads, one write): y = x + z elementwise over FP64 values; x, z and y are
 * device buffers of `bytes` each (a multiple of 16, 16-byte aligned), y may
 * alias neither input.  PV_ERR_INVALID_ARG on a null or misaligned pointer
 * or size. */
pv_status pv_stream_triad(const void *x, const void *z, void *y, size_t bytes, void *stream);

/* Third bandwidth reference, reads only: every 16-byte chunk of x (a device
 * buffer of `bytes`, a multiple of 16, 16-byte aligned) is loaded once and
 * folded into a 32-bit XOR per wave, written to `sink` (a device buffer of
 * PV_STREAM_READ_SINK_BYTES, caller-owned; its contents are a checksum with
 * no other meaning).  PV_ERR_INVALID_ARG on a null or misaligned pointer or
 * size. */
#define PV_STREAM_READ_SINK_BYTES 65536
pv_status pv_stream_read(const void *x, size_t bytes, void *sink, void *stream);

/*
 * Launch shape of the stencil sweep for one (dtype, nb) of a lattice -- the
 * GPU counterpart of the cache-blocking choices of Sec. 3.1 (layer
 * conditions, blocking factor).  Zero fields take the library's defaults.
 *   kernel           0 choose, 1 direct (every neighbour load goes through the
 *                    caches; any stencil), 2 staged (LDS ring of rows along
 *                    the outer lattice axis; compiled stencil families, and
 *                    generic 3D stencils with no offset that has both a y
 *                    and a z step, with 16-byte aligned blocks; otherwise
 *                    direct is used)
 *   elems_per_lane   staged: 1 or 2 (complex128), 2 or 4 (complex64)
 *   walk_planes      staged: outer-axis planes per walk of a workgroup
 *   strip_rows       staged: middle-axis rows per strip of the work order
 *   groups_per_xcd   staged: workgroups per XCD, 1..256
 *   tiles_per_group  direct: row tiles per workgroup, up to 64 (values below
 *                    the default are raised to it)
 *   slab_rows        direct: y rows per slab of the sweep order
 *   workgroup_size   staged: lanes per workgroup, 256 (0: default) or 512
 *                    (a tile twice as long: half the relative x halo;
 *                    compiled stencil families, the Chebyshev, series and
 *                    plain sweeps)
 * The shape changes speed only: every shape computes the same result up to
 * the summation order of the fused dot products.
 */
typedef struct pv_tuning {
    int kernel;
    int elems_per_lane;
    int walk_planes;
    int strip_rows;
    int groups_per_xcd;
    int tiles_per_group;
    int slab_rows;
    int workgroup_size;
} pv_tuning;

/* Set (t != NULL) or reset to defaults (t == NULL) the shape used for
 * (dtype, nb), by every sweep including series steps (this drops a series
 * shape the autotuner chose); get returns the shape of the Chebyshev step.
 * PV_ERR_INVALID_ARG for values outside the ranges above. */
pv_status pv_lattice_set_tuning(pv_lattice *lat, int dtype, int nb, const pv_tuning *t);
pv_status pv_lattice_get_tuning(const pv_lattice *lat, int dtype, int nb, pv_tuning *t);

/*
 * Generated stencil kernels (Sec. 3.2: the DSL front end generates the code
 * of a model's stencil).  A stencil that none of the built-in families
 * matches (PV_FAM_GENERIC: any DSL program or descriptor) is described at
 * lattice creation as a pattern struct -- its offsets in descriptor order
 * and, for every block entry, whether it is zero, real, imaginary or complex
 * -- and its sweeps take the built-in families' staged and direct kernels
 * instantiated for that pattern, compiled with hipRTC for the current
 * device on the first launch that needs an instance (about a second each;
 * the code objects stay loaded until the process ends, and PV_CODEGEN_CACHE
 * may name a directory that keeps them across processes).  Compile on a
 * launch outside stream capture first: compilation is not a stream operation.
 * Results equal the interpreted generic kernels' up to the summation order
 * of the stencil terms.  3D stencils with an offset that has both a y and a
 * z step take the direct kernel, others the staged one as the built-in
 * families do (with 512-lane workgroups available to the autotuner).
 * A failed compilation returns PV_ERR_HIP with the compiler's log in
 * pv_last_error() (for tests, PV_TEST_FAIL_CODEGEN=1 in the environment
 * makes every compilation fail); the lattice stays usable.  Batched sweeps (pv_batch_*) take generated kernels when
 * all their lattices share one pattern.
 *
 * set_codegen: enable (1, the default) or disable (0: the interpreted
 * generic kernels, which read every entry's column and value at run time)
 * for this lattice; PV_CODEGEN=0 in the environment disables it for every
 * lattice.  get_codegen: *active = 1 when sweeps of the lattice take
 * generated kernels (a generic stencil with a pattern, enabled).
 * codegen_source: the pattern struct's C++ text, NUL-terminated into buf
 * (truncated to len - 1 bytes; buf may be NULL), *needed (may be NULL) =
 * its length + 1; PV_ERR_UNSUPPORTED for built-in families and for stencils
 * whose block rows need more than 96 per-lane entry slots (those always take
 * the interpreted kernels).
 */
pv_status pv_lattice_set_codegen(pv_lattice *lat, int enable);
pv_status pv_lattice_get_codegen(const pv_lattice *lat, int *active);
pv_status pv_lattice_codegen_source(const pv_lattice *lat, char *buf, size_t len, size_t *needed);
/* Number of generated kernel instances compiled (or read from the cache) and
 * loaded in this process, over all devices: an instance is one kernel for
 * one pattern, launch shape and epilogue. */
int pv_codegen_instances(void);

/*
 * Autotuner: times candidate shapes of one Chebyshev step (sweep with fused
 * dots and its reduction) on the stream's device and applies the fastest to
 * the lattice for (dtype, nb); then, separately, those of one series step
 * (the accumulating sweep of pv_cheb_series, pv_cheb_propagate, pv_chebfd
 * and pv_trlanczos_fd, whose extra stream changes the best shape), applied
 * to that step only.  cache_path names a JSON-lines file (NULL:
 * the PV_TUNE_CACHE environment variable, else no cache); an entry whose key
 * (stencil family, orbitals, extents, boundary conditions, nb, dtype, field
 * type, device architecture and CU count) matches is applied without timing,
 * and a new result is appended.  work: pv_autotune_workspace_size() bytes,
 * overwritten.  Synchronises the stream.  out and ms (either may be NULL)
 * receive the chosen shape and its time per step in milliseconds (0 when
 * the shape came from the cache).
 */
size_t pv_autotune_workspace_size(const pv_lattice *lat, int dtype, int nb);
pv_status pv_autotune(pv_lattice *lat, int dtype, int nb, const char *cache_path, void *work,
                      size_t work_bytes, void *stream, pv_tuning *out, double *ms);

/*
 * Launch shape of a batch (pv_batch_kpm_moments) for (dtype, nb): the
 * kernel, elements per lane and lanes per workgroup of pv_tuning (other
 * fields are ignored: each instance walks whole columns of its lattice with
 * workgroups of its own).  Unset, a batch takes lattice 0's kernel and
 * elements per lane with 256-lane workgroups.  Setting or resetting (t ==
 * NULL) drops the captured graph.  512-lane workgroups need a compiled
 * stencil family or generated kernels (PV_ERR_UNSUPPORTED otherwise).  A
 * batch of generic-stencil lattices takes generated kernels (compiled
 * before its graph is captured) when every lattice has them enabled and
 * all share one pattern; otherwise the interpreted direct kernel.
 *
 * pv_batch_autotune times the candidate shapes -- the direct kernel; the
 * staged kernel with each elements-per-lane value and 256 or 512 lanes --
 * each on a captured run of the batch itself (8 Chebyshev steps of every
 * instance with start blocks r and scales a, b as for pv_batch_kpm_moments,
 * timed as the fastest of three replays), and keeps the fastest for the
 * batch.  work: pv_batch_autotune_workspace_size() bytes (the largest
 * over the candidate shapes, whatever shape the batch holds), overwritten.
 * Synchronises the stream.  out and ms (either may be NULL) receive the
 * chosen shape and its time per batched step in milliseconds.
 */
pv_status pv_batch_set_tuning(pv_batch *batch, int dtype, int nb, const pv_tuning *t);
pv_status pv_batch_get_tuning(const pv_batch *batch, int dtype, int nb, pv_tuning *t);
size_t pv_batch_autotune_workspace_size(const pv_batch *batch, int dtype, int nb);
pv_status pv_batch_autotune(pv_batch *batch, int dtype, int nb, const double *a, const double *b,
                            const void *const *r, void *work, size_t work_bytes, void *stream,
                            pv_tuning *out, double *ms);

#ifdef __cplusplus
}
#endif
#endif /* PVDTM_H */

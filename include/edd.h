/*
 * edd.h -- C ABI of the MI355X Schur-interface elasticity solver.
 *
 * The library solves the discrete isotropic linear-elasticity system
 * K(E) u = f of Turner, Kocvara and Loghin (arXiv 1501.06211), Section 2,
 * eq. (NumberFour), on a structured grid of unit Q1 quadrilaterals (2D,
 * plane stress) or trilinear hexahedra (3D), by the non-overlapping domain
 * decomposition of Section 1: interior unknowns of every subdomain are
 * eliminated with batched direct solves (K_II is the direct sum of the
 * subdomain blocks, eq. (NumberFive)) and the interface (Schur complement)
 * system S u_G = f_G - K_GI K_II^{-1} f_I of eq. (3MatSplit) is solved by a
 * preconditioned Krylov method, optionally with the interface preconditioner
 * Hhat_theta of Section 3, eqs. (NumberEight)-(NumberNine).
 *
 * Conventions used by every entry point
 *   - Node (i,j[,k]) has id i + (nx+1)*(j + (ny+1)*k); element (ex,ey[,ez])
 *     has id ex + nx*(ey + ny*ez) (x fastest).
 *   - Nodal vectors are node-major with components interleaved: entry
 *     dim*node + c.  All public vectors are FP64 device pointers.
 *   - "Gamma" vectors hold the interface dofs, nodes in increasing id order,
 *     components interleaved: length dim * n_gamma.
 *   - "Interior" vectors hold the interior dofs packed subdomain by
 *     subdomain in the library's own local order; edd_get_interior_nodes
 *     gives that order.
 *   - Every call is asynchronous on the stream given to edd_setup_mesh
 *     unless it says it synchronises.  A handle is used by one host thread
 *     at a time.  The caller owns every *_dev buffer and the stream; the
 *     library owns the handle and all memory it allocates (through the
 *     allocator given at setup, or hipMalloc when that is NULL) and frees
 *     it in edd_destroy.
 *   - Return values: EDD_OK (0), EDD_NOT_CONVERGED (1, results valid), or a
 *     negative error code; no C++ exception crosses this interface.
 */
#ifndef EDD_H
#define EDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ----------------------------------------------------- */
#define EDD_OK 0
#define EDD_NOT_CONVERGED 1
#define EDD_EINVAL (-1)     /* bad argument (sizes, NaN/Inf, E <= 0, ...)   */
#define EDD_ENOMEM (-2)     /* device allocation failed                     */
#define EDD_EHIP (-3)       /* a HIP call failed; see edd_last_hip_error    */
#define EDD_ESTATE (-4)     /* call out of order (e.g. solve before moduli) */
#define EDD_ENOTSPD (-5)    /* a pivot of an interior factor was <= 0       */
#define EDD_EBREAKDOWN (-6) /* Krylov breakdown (p^T S p <= 0, NaN, ...)    */

/* ---- enumerations ----------------------------------------------------- */
#define EDD_F64 1 /* dtype / factor precision bits */
#define EDD_F32 2

#define EDD_CLAMP_X0 1 /* clamped faces (u = 0 on the Dirichlet boundary) */
#define EDD_CLAMP_X1 2
#define EDD_CLAMP_Y0 4
#define EDD_CLAMP_Y1 8
#define EDD_CLAMP_Z0 16
#define EDD_CLAMP_Z1 32

#define EDD_MODE_F64 0   /* everything in FP64                               */
#define EDD_MODE_MIXED 1 /* iterative refinement of the interface problem:   */
                         /* FP64 residuals, inner solves with FP32 factors  */
#define EDD_MODE_RELAXED 2 /* one flexible CG whose S applies switch from    */
                           /* FP64 to FP32 factors once the residual is     */
                           /* below mixed_inner_tol times the initial one   */
                           /* (inexact Krylov with relaxed accuracy)        */

#define EDD_PC_IDENTITY 0 /* S~ = I                                           */
#define EDD_PC_HTHETA 1   /* S~ = Hhat_theta by inverse Lanczos (Section 3)   */
#define EDD_PC_SCHUR 2    /* S~ = S itself, applied by an inner interface     */
                          /* solve to mixed_inner_tol (edd_solve_gmres only)  */

/* edd_solve_opts.pc_form (Section 3, eqs. (NumberEight)-(NumberNine)):
 * Htilde_theta = M (M^{-1} L)^{1-theta} or H_theta = M + M (M^{-1} L)^{1-theta}
 * per component, applied by inverse Lanczos on L^{-1} M (every step an inner
 * face-block PCG on L) or by forward ("truncated") Lanczos on M^{-1} L (every
 * step one product with L, no inner solves).  H_theta needs no inverse of L,
 * so its forward form also serves skeletons that do not meet the clamp. */
#define EDD_PCF_HTILDE_INV 0 /* Htilde_theta, inverse Lanczos (default)       */
#define EDD_PCF_H_INV 1      /* H_theta, inverse Lanczos                      */
#define EDD_PCF_HTILDE_FWD 2 /* Htilde_theta, forward Lanczos                 */
#define EDD_PCF_H_FWD 3      /* H_theta, forward Lanczos                      */

/* stats.flags bits */
#define EDD_FLAG_TRUE_RES_RESTART 1 /* recursive residual disagreed; restarted */
#define EDD_FLAG_MIXED_FALLBACK 2   /* mixed path stalled; fell back to FP64   */
#define EDD_FLAG_PC_DROPPED 4       /* reserved: never set (a step without     */
                                    /* descent ends the solve, EDD_EBREAKDOWN) */
#define EDD_FLAG_LEARNED_REJECTED 8 /* a network proposal was dropped: its      */
                                    /* interface energy <d,Sd> was not positive */

typedef struct edd_problem edd_problem;

/* Device memory callbacks.  alloc returns NULL on failure. */
typedef struct edd_allocator {
  void *(*alloc)(void *ctx, size_t bytes);
  void (*free)(void *ctx, void *ptr);
  void *ctx;
} edd_allocator;

/* Geometry of one problem (host memory, read during the call only). */
typedef struct edd_mesh_desc {
  int dim;              /* 2 or 3                                            */
  int nel[3];           /* elements per axis; nel[2] ignored when dim == 2   */
  int ncuts[3];         /* entries of cuts[a] (subdomain blocks + 1)         */
  const int *cuts[3];   /* increasing cut positions, cuts[a][0] = 0 and      */
                        /* cuts[a][ncuts[a]-1] = nel[a]; blocks may differ   */
  double nu;            /* Poisson ratio, -1 < nu < 1/2 (Section 1)          */
  int clamp_faces;      /* EDD_CLAMP_* bitmask; at least one face            */
  int factor_precision; /* EDD_F64 and/or EDD_F32: which interior factors    */
                        /* edd_set_element_moduli builds                     */
  int dissect;          /* 3D interior solves: split a subdomain's interior  */
                        /* into two band blocks and a separator plane (one  */
                        /* level of nested dissection) so that more         */
                        /* workgroups share its substitution; -1: when its  */
                        /* band work exceeds 1.5x the median, or when there */
                        /* are fewer subdomains than compute units (then    */
                        /* every interior of >= 3000 dofs), 0: never, 1:    */
                        /* every interior with at least 5 planes, 2: only   */
                        /* interiors above 1.5x the median band work; 2D    */
                        /* problems never split                             */
} edd_mesh_desc;

typedef struct edd_solve_opts {
  double tol;         /* stop when ||f - K u||_2 <= tol * ||f||_2 (free dofs) */
  int maxit;          /* max interface iterations (per inner solve if mixed)  */
  int precision;      /* EDD_MODE_F64 or EDD_MODE_MIXED                       */
  int precond;        /* EDD_PC_IDENTITY or EDD_PC_HTHETA                     */
  double theta;       /* H_theta index in [0,1]; < 0 picks the value reported  */
                      /* best for the number of subdomains (0.5 at 4, 0.6 at */
                      /* 16, 0.7 at 64, 0.75 from 256, log-linear between)   */
  int lanczos_kmax;   /* max inverse-Lanczos steps per application (<= 64)   */
  double lanczos_tol; /* relative change that stops Lanczos early            */
  double inner_tol;   /* relative tolerance of the skeleton-Laplacian PCG    */
  int inner_maxit;    /* max iterations of that PCG                          */
                      /* lanczos_tol <= 0 and inner_tol <= 0 select the     */
                      /* device-resident form: exactly lanczos_kmax (<= 32) */
                      /* steps of inner_maxit iterations, no host waits     */
  int use_initial_guess; /* u_dev holds an initial guess on entry             */
  int outer_maxit;    /* mixed mode: max refinement rounds                   */
  double mixed_inner_tol; /* EDD_MODE_MIXED: relative tolerance of each      */
                          /* round's FP32-factor interface solve;            */
                          /* EDD_MODE_RELAXED: relative residual at which    */
                          /* the S applies switch to FP32 factors            */
  int flexible_window; /* directions kept by the flexible Krylov (0 = all,   */
                       /* up to 8192, or 256 for the captured iteration;    */
                       /* 1 = short recurrence).  They are stored in blocks */
                       /* of 256 vectors of 2 n_gamma dim doubles (the      */
                       /* direction and its S image), allocated when the    */
                       /* iteration first reaches them and kept until       */
                       /* edd_destroy                                       */
  int interface_weighting; /* 0: M, L of the skeleton as in the paper;        */
                           /* 1: each skeleton element scaled by the mean     */
                           /*    modulus of its two neighbouring elements     */
  int learned_guess;  /* 1: add the correction network's proposal to the     */
                      /* initial guess, scaled by the exact minimiser of the */
                      /* interface energy error along it (needs              */
                      /* edd_cnn_setup); 0: off                              */
  int use_graphs;     /* 1: the device-resident preconditioner apply is      */
                      /* captured once into a HIP graph and replayed;        */
                      /* n >= 2: the interface iteration itself runs as      */
                      /* replays of a captured graph of n iterations (up to  */
                      /* 64; device-resident preconditioner, FP64 or mixed   */
                      /* mode, a window of at most 256 directions; a larger  */
                      /* one runs the host-driven loop): the window comes    */
                      /* from a device iteration                             */
                      /* index and a device flag marks convergence, read by  */
                      /* the host once per replay.  Up to the first         */
                      /* converged iteration the arithmetic is bitwise that  */
                      /* of the host-driven loop, which checks every 4       */
                      /* iterations; the steps a replay runs after that only */
                      /* refine u.  Kernel timing is not recorded inside the */
                      /* graph.                                              */
  int pc_form;        /* EDD_PCF_*: which interface norm S~ applies and how  */
  int learned_correction; /* K > 0: every K-th interface step takes its      */
                      /* direction from the correction network applied to the */
                      /* interface residual extended by zero instead of S~;   */
                      /* a step without a usable direction is dropped (flag   */
                      /* EDD_FLAG_LEARNED_REJECTED); needs edd_cnn_setup;     */
                      /* 0: off                                               */
  int mass_matrix;    /* skeleton mass matrix M of the interface norm        */
                      /* (Section 3): 0 lumped (row sums, diagonal: M^{-1}  */
                      /* and the M inner products are exact scalings), 1    */
                      /* the consistent FE mass matrix (its products are    */
                      /* sparse products in the pattern of L; M^{-1} by     */
                      /* Chebyshev iteration on the Jacobi-scaled M, whose  */
                      /* spectrum the element matrices bound: [1/2, 3/2]    */
                      /* in 2D, [1/4, 9/4] in 3D, to 1e-12)                  */
} edd_solve_opts;

typedef struct edd_solve_stats {
  int status;
  int iterations;           /* interface Krylov iterations (all inner solves) */
  int outer_iterations;     /* refinement rounds (mixed mode), else 0         */
  int precond_applications;
  int lanczos_steps;        /* total inverse-Lanczos steps                    */
  int inner_iterations;     /* total skeleton-Laplacian PCG iterations        */
  int flags;                /* EDD_FLAG_* bits                                */
  double rel_residual;      /* final ||f - K u|| / ||f|| from an FP64 K apply */
  double compliance;        /* f^T u (eq. (NumberTen))                        */
  double t_total_ms;        /* wall time of the call                          */
  double t_krylov_ms;       /* interface iteration part                       */
  double learned_alpha;     /* step taken along the network's proposal (0 if  */
                            /* off or rejected)                               */
} edd_solve_stats;

typedef struct edd_info {
  int dim, n_sub;
  int64_t n_nodes, ndof, n_el;
  int64_t n_gamma;          /* interface nodes                                */
  int64_t n_interior_dofs;  /* length of interior vectors                     */
  int64_t factor_entries;   /* band entries of all K_{I_i I_i} (no padding)   */
  int max_band;             /* largest half bandwidth                         */
  int max_sub_dofs;         /* largest subdomain interior size                */
  int64_t skeleton_faces;   /* face blocks of the interface preconditioner    */
  int face_classes;         /* distinct face-block shapes                     */
  double theta_default;
  int band_blocks;          /* band blocks after dissection (>= n_sub)         */
  int64_t coupling_entries; /* entries of the dissection couplings W_h         */
} edd_info;

/* Fill *o with the defaults: tol 1e-8, maxit 2000, FP64, Hhat_theta with
 * theta 0.5 in the device-resident form with 3 Lanczos steps of 4 inner
 * iterations (the fastest such pair on a 1.6M-dof 3D cantilever; the
 * paper's adaptive form is lanczos_tol 1e-2, inner_tol 1e-3, Section 4), no initial guess, outer_maxit 20, mixed_inner_tol 1e-4,
 * flexible_window 0, interface_weighting 1, learned_guess 0, use_graphs 0. */
void edd_default_opts(edd_solve_opts *o);

/* Build a problem handle from the grid, the subdomain cuts, nu and the
 * clamped faces (Section 1: nodes shared by two or more subdomain closures
 * form Gamma, clamped nodes are removed, all others are interior to one
 * subdomain).  Does the host-side bookkeeping, uploads the maps and builds
 * the geometry-only parts of the interface preconditioner.  hip_stream is
 * a hipStream_t (NULL = default stream).  On success *out owns all library
 * memory.  Synchronises. */
int edd_setup_mesh(const edd_mesh_desc *d, const edd_allocator *a,
                   void *hip_stream, edd_problem **out);

/* Set the element moduli E_e (n_el values on the device, element order as
 * above; dtype EDD_F64 or EDD_F32): K(E) = sum_e E_e K0_e, the linear
 * dependence of eq. (NumberTen).  Assembles the interior blocks K_{I_i I_i}
 * and factors them (band Cholesky) in the precision(s) chosen at setup.
 * Returns EDD_EINVAL if any E_e is not finite and positive, EDD_ENOTSPD if
 * a pivot is not positive.  Synchronises (to report those errors). */
int edd_set_element_moduli(edd_problem *p, const void *E_dev, int dtype);

/* y = K(E) u over all dofs (Section 2, eq. (NumberFour)).  Clamped entries
 * of u are ignored (treated as 0) and clamped entries of y are set to 0.
 * u_dev and y_dev must not overlap.  Requires moduli. */
int edd_apply_K(edd_problem *p, const double *u_dev, double *y_dev);

/* Solve K u = f on the free dofs by the three steps of eq. (3MatSplit):
 * condensation, preconditioned Krylov on S u_G = g, back-substitution.
 * u_dev receives the full-length solution (0 on clamped dofs); on entry it
 * is the initial guess if o->use_initial_guess.  s may be NULL.
 * Synchronises.  Returns EDD_NOT_CONVERGED (u valid, best iterate) when
 * the tolerance is not met within the iteration limits. */
int edd_solve_interface(edd_problem *p, const double *f_dev, double *u_dev,
                        const edd_solve_opts *o, edd_solve_stats *s);

/* Solve K u = f on the free dofs by the paper's own Krylov method (Section
 * 3): flexible GMRES on the whole system, preconditioned from the right by
 * the block-triangular P~ = [K_II K_IG; 0 S~], whose inverse is applied in
 * the factored order printed there (S~^{-1} on the interface part, then the
 * interior part K_II^{-1} (v_I - K_IG z_G)).  S~ is o->precond: EDD_PC_IDENTITY,
 * EDD_PC_HTHETA (settings as for edd_solve_interface) or EDD_PC_SCHUR (S
 * itself by an inner interface solve to relative tolerance
 * o->mixed_inner_tol; GMRES then needs at most two iterations).  Stops when
 * the GMRES residual is <= tol ||f||, then checks the FP64 true residual and
 * restarts from u if it misses.  o->flexible_window is the restart length
 * (0: 256, at most 256); o->maxit bounds the GMRES iterations; stats report
 * them in `iterations`, and the inner interface iterations of EDD_PC_SCHUR
 * (at most 5000 per application) in `outer_iterations`.  Synchronises. */
int edd_solve_gmres(edd_problem *p, const double *f_dev, double *u_dev,
                    const edd_solve_opts *o, edd_solve_stats *s);

/* ---- parts of the path, exposed for checking and for composition ------ */

/* x = K_II^{-1} b on interior vectors (eq. (3MatSplit2), first and third
 * lines), with the factor of precision EDD_F64 or EDD_F32.  b and x may be
 * the same buffer. */
int edd_solve_interior(edd_problem *p, const double *b_dev, double *x_dev,
                       int precision);

/* y = S v on Gamma vectors, S = K_GG - K_GI K_II^{-1} K_IG (Section 2),
 * with the interior factor of the given precision. */
int edd_apply_S(edd_problem *p, const double *v_dev, double *y_dev,
                int precision);

/* z = S~^{-1} r on Gamma vectors for the preconditioner chosen in *o
 * (Section 3).  Synchronises when the preconditioner is Hhat_theta. */
int edd_apply_precond(edd_problem *p, const double *r_dev, double *z_dev,
                      const edd_solve_opts *o);

/* Pieces of the interface preconditioner on Gamma vectors (all d
 * components), for checking and composition (Section 3 and Section 4):
 *   which 0: y = L x     (skeleton Laplacian, weighting as requested)
 *   which 1: y = M x     (lumped skeleton mass)
 *   which 2: y = B^{-1} x (L restricted to the faces, cross points removed)
 *   which 3: y ~ L^{-1} x by PCG with B (relative tolerance tol, maxit)
 *   which 4: y = M x     (consistent skeleton mass)
 *   which 5: y ~ M^{-1} x (consistent mass, the Chebyshev iteration of the
 *            mass_matrix = 1 preconditioner)
 * weighting as edd_solve_opts.interface_weighting (1 needs moduli).
 * Synchronises for which 3. */
int edd_apply_skeleton_op(edd_problem *p, int which, int weighting,
                          const double *x_dev, double *y_dev, double tol,
                          int maxit);

/* ---- allocation-free variant -------------------------------------------
 * For callers that cannot allocate device memory while they run: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * edd_apply_S_noalloc computes y = S v exactly as edd_apply_S (same kernels,
 * same order, bitwise equal results), but its interior-length work vector
 * lives in one static device array of EDD_NOALLOC_MAX_INTERIOR_DOFS doubles
 * (16 MiB) that every GPU the library runs on holds until the process ends,
 * instead of the handle's own buffer.  The call allocates nothing and makes
 * no allocating library call (kernel timing is suspended for its duration).
 * The handle must come from edd_setup_mesh (which looks up the array's
 * address on its device) and have moduli set.
 * Errors: EDD_EINVAL for NULL pointers, a bad precision, or an interior
 * vector longer than EDD_NOALLOC_MAX_INTERIOR_DOFS (edd_info.
 * n_interior_dofs); EDD_ESTATE before moduli or without factors of that
 * precision.  Every call on one GPU shares that GPU's array, which keeps the
 * last call's contents (they are never read): calls that overlap on one GPU
 * (several streams or host threads) race, and the caller must serialise them. */
#define EDD_NOALLOC_MAX_INTERIOR_DOFS (1 << 21)
int edd_apply_S_noalloc(edd_problem *p, const double *v_dev, double *y_dev,
                        int precision);

/* ---- many problems and tile shapes ------------------------------------ */

/* Solve n independent problems concurrently: a pool of nthreads host
 * threads (<= 0: 16) drives the handles, each on its own stream, so the
 * GPU overlaps their kernels.  The handles must be distinct and should be
 * created on distinct streams (one stream serialises them).  stats (n
 * entries) may be NULL; each entry's t_total_ms is that problem's latency.
 * Returns the first error, else EDD_NOT_CONVERGED if any problem missed
 * the tolerance, else EDD_OK. */
int edd_solve_batch(edd_problem *const *ps, int n, const double *const *f_dev,
                    double *const *u_dev, const edd_solve_opts *o,
                    edd_solve_stats *stats, int nthreads);

/* Autotuner of the tile shapes:
 *  - the batched interior substitution: every variant valid for this
 *    problem's bands (1-3: one row per thread with an owner wavefront per
 *    diagonal block, 64/256/512 threads per subdomain; 4-6: wide bands, a
 *    dedicated chain wavefront and 1024 threads, two load chunk widths, the
 *    narrower one also double-buffered; 7: as 6 with lookahead, the chain
 *    wavefront applying the previous block to its own rows while the others
 *    apply it to the rows below), for FP64 and (if present) FP32 factors,
 *    timed on the current factors;
 *  - the element kernel: node tiles of 16x16 / 32x8 / 64x4 (2D) or 8x8x4 /
 *    16x4x4 / 16x8x2 (3D) nodes (every shape gives bitwise the same result),
 *    chosen separately for the full product, the product on interior nodes
 *    and the product on interface nodes (the two halves of an S apply);
 *  - the S apply (edd_set_s_apply): explicit local Schur complements where
 *    the problem allows them, if their FP64 apply is faster (the choice is
 *    applied to the handle; edd_get_s_apply reports it).
 * The fastest of each is kept.  Choices are cached per (device
 * architecture, kernel family, shape class: dimension, band extents and
 * factor precisions for the substitution, the node grid for the element
 * kernel) in memory for the process and, after edd_autotune_cache, in that
 * file; force != 0 re-times.  variants (5 ints: FP64 and FP32 substitution
 * variants, element tile shapes for all / interior / interface nodes) may
 * be NULL.  Needs edd_set_element_moduli.
 * Synchronises. */
int edd_autotune(edd_problem *p, int force, int *variants);
/* Use (and create or update) the autotuner cache file at path (NULL or "":
 * memory only): loads the file's entries, replacing the in-memory cache.
 * Text, one line per entry: family, key, values.  Not thread-safe against
 * concurrent edd_autotune calls in other threads. */
int edd_autotune_cache(const char *path);
/* Choose the substitution variants by hand (0 = default by bandwidth). */
int edd_set_solve_variants(edd_problem *p, const int *variants);
/* How S v is applied (the Steklov-Poincare splitting S = sum_i R_i^T S_i R_i
 * over the subdomains, Section 1; the subdomain problems of eq.
 * (3MatSplit2)):
 *   0  through the interior factors: S v = (K[-K_II^{-1}(K[0;v])_I ; v])_G
 *      (the default);
 *   1  explicit local Schur complements S_i = K^i_GG - K^i_GI (K^i_II)^{-1}
 *      K^i_IG on the interface dofs of each subdomain's closure (its own
 *      elements), formed on the device after every edd_set_element_moduli
 *      from the FP64 interior factors (a forward substitution with all
 *      right-hand sides, then K^i_GG - Y^T Y), stored dense (sum_i m_i^2
 *      doubles) and applied as one dense matrix-vector product per
 *      subdomain plus a fixed-order sum over the subdomains of each
 *      interface dof.
 * Mode 1 serves FP64 applies (FP32 applies of the mixed modes keep mode 0)
 * and needs undissected interiors, FP64 factors and m_i <= 1024 with the
 * formation's LDS ring fitting one workgroup: EDD_EINVAL otherwise (2D
 * decompositions qualify; 3D ones only with small subdomains).  The
 * element-kernel timings (edd_get_kernel_times) do not include it.
 * Synchronises when it forms S_i. */
int edd_set_s_apply(edd_problem *p, int mode);
int edd_get_s_apply(edd_problem *p, int *mode);
/* Choose the element kernel's node-tile shape by hand (0..2, as above) for
 * all three kinds of target. */
int edd_set_apply_variant(edd_problem *p, int variant);

/* ---- correction network (an addition to the paper's method) -----------
 * A convolution network on the node grid proposes a displacement correction
 * d ~ K^{-1} r from a stiffness indicator (per node, the mean over adjacent
 * elements of clip(1 + log10(E_e)/3, 0, 1)) and the residual r divided by
 * its root mean square over free dofs.  Four layers of 3^dim taps with
 * dilations 1, 2, 4, 1 and ReLU after the first three; widths 1+dim -> 32
 * -> 32 -> 32 -> dim.  Activations are node-major FP32, the forward pass
 * uses FP16 weights with FP32 accumulation, and the master weights are
 * FP32, trained by Adam (beta 0.9/0.999, eps 1e-8) on the relative squared
 * L2 loss against e / rms(e).  Parameters are one flat FP32 array: per
 * layer W[tap][c_in][c_out] (taps in C order over the ([z,] y, x) offsets
 * -1, 0, 1 times the dilation) followed by b[c_out].
 * The solver uses the proposal only through edd_solve_opts.learned_guess. */

/* Allocate the network for this problem; width must be 32.  Parameters
 * start at zero. */
int edd_cnn_setup(edd_problem *p, int width);
/* 1: run the forward pass of the two hidden 32 -> 32 layers on the FP16
 * matrix cores (implicit GEMM by v_mfma_f32_16x16x16_f16: FP16 weights and
 * FP16-rounded activations, FP32 accumulation; relative error against the
 * FP32 path about 1e-3), for inference and training alike; 0 (default):
 * the FP32 vector path.  Needs edd_cnn_setup. */
int edd_cnn_matrix_cores(edd_problem *p, int enable);
/* Number of FP32 parameters. */
int edd_cnn_num_params(edd_problem *p, int64_t *n);
/* Copy device parameters in (resets the Adam moments) or out. */
int edd_cnn_set_params(edd_problem *p, const float *params_dev);
int edd_cnn_get_params(edd_problem *p, float *params_dev);
/* d = network(E, r) on full-length nodal vectors; d is zero at Dirichlet
 * dofs.  E_dev: n_el FP64 element moduli for the stiffness indicator, or
 * NULL for the moduli set last (these need not be the factored ones). */
int edd_cnn_predict(edd_problem *p, const double *E_dev, const double *r_dev,
                    double *d_dev);
/* Loss and its gradient (FP32, parameter layout) for the pair (r, e), where
 * e is the correction that r calls for; grad_dev may be NULL.  No update. */
int edd_cnn_loss_grad(edd_problem *p, const double *E_dev, const double *r_dev,
                      const double *e_dev, float *grad_dev, double *loss);
/* One Adam step with learning rate lr on the pair (r, e); *loss receives
 * the loss before the step. */
int edd_cnn_train_step(edd_problem *p, const double *E_dev, const double *r_dev,
                       const double *e_dev, double lr, double *loss);

/* Training pair of one warm-started step of a moduli sequence: with the
 * moduli of step k set, r = f - K(E_k) u_prev (zero on clamped dofs) is the
 * residual the warm start leaves, and e = u - u_prev the correction that
 * the solve u of step k applied to it.  Full-length nodal vectors; r and e
 * must not alias u_prev, u or each other (f may alias nothing written).
 * Requires moduli. */
int edd_cnn_training_pair(edd_problem *p, const double *f_dev,
                          const double *u_prev_dev, const double *u_dev,
                          double *r_dev, double *e_dev);

/* Sizes of the problem. */
int edd_get_info(edd_problem *p, edd_info *info);

/* Host copies of the node ids behind Gamma vectors (n_gamma entries) and
 * behind interior vectors (n_interior_dofs / dim entries, one per node). */
int edd_get_gamma_nodes(edd_problem *p, int32_t *nodes_host);
int edd_get_interior_nodes(edd_problem *p, int32_t *nodes_host);

/* ---- topology optimisation (Section 5) -----------------------------------
 * The fixed-point loop of Section 5 for min f^T u subject to K(rho) u = f,
 * K(rho) = sum_i E(rho_i) K0_i (eq. (NumberTen)), sum_i rho_i <= V and
 * rho_min <= rho_i <= rho_max: finite element analysis (edd_solve_interface),
 * an Optimality Criteria density update, a convergence check.  With
 * penal = 1 and emin = 0, E(rho) = rho: the paper's Variable Thickness
 * Sheet problem; otherwise E(rho) = emin + rho^penal (1 - emin).
 * Densities are FP64 device vectors of n_el values in element order. */

typedef struct edd_oc_params {
  double volume;           /* V, the bound on sum_i rho_i                     */
  double rho_min, rho_max; /* box bounds, 0 < rho_min <= rho_max              */
  double move;             /* move limit |rho_new - rho| <= move              */
  double eta;              /* damping exponent of the OC fixed point          */
  double penal, emin;      /* E(rho) as above (penal >= 1, 0 <= emin < 1)     */
} edd_oc_params;

typedef struct edd_oc_result {
  double lambda;     /* multiplier of the volume constraint (0: the bound was */
                     /* not reached with every density at its upper limit;  */
                     /* +inf: the lower limits already exceed it)           */
  double volume;     /* sum of the new densities                              */
  double max_change; /* max_i |rho_new_i - rho_i|                             */
} edd_oc_result;

/* s_e = u_e^T K0 u_e for every element: twice the strain energy of the
 * element at unit modulus, -dc/dE_e (clamped dofs of u count as zero).
 * u_dev: full nodal vector; s_dev: n_el values.  Asynchronous. */
int edd_element_energies(edd_problem *p, const double *u_dev, double *s_dev);

/* One OC update: with g_i = E'(rho_i) s_i,
 *   rho_new_i = clamp(rho_i (g_i / Lambda)^eta, max(rho_min, rho_i - move),
 *                     min(rho_max, rho_i + move)),
 * Lambda found on the device so that sum_i rho_new_i = V (multisection on
 * log Lambda to a relative width below 1e-11).  E_new_dev (may be NULL)
 * receives E(rho_new).  rho_new_dev must not alias rho_dev or s_dev.
 * Returns EDD_EINVAL for bad parameters.  Synchronises. */
int edd_oc_update(edd_problem *p, const double *rho_dev, const double *s_dev,
                  const edd_oc_params *o, double *rho_new_dev, double *E_new_dev,
                  edd_oc_result *res);

typedef struct edd_topopt_opts {
  double volfrac;            /* V = volfrac * n_el                            */
  double rho_min, rho_max, move, eta, penal, emin;  /* as edd_oc_params       */
  double change_tol;         /* stop when max |rho_new - rho| <= change_tol   */
  int maxit;                 /* fixed-point iterations at most                */
  int adaptive_tol;          /* 1: Krylov tolerance of step k is             */
                             /* |c_{k-1} - c_{k-2}| / c_{k-1} clamped to     */
                             /* [tol_min, tol_max] (tol_max for the first    */
                             /* two steps); 0: tol_min throughout            */
  double tol_min, tol_max;
  int warm_start;            /* 1: each analysis starts from the previous u  */
} edd_topopt_opts;

typedef struct edd_topopt_stats {
  int status;                /* EDD_OK, or EDD_NOT_CONVERGED if an analysis  */
                             /* missed its tolerance                         */
  int steps;                 /* fixed-point iterations done                  */
  int converged;             /* 1 if the change test was met                 */
  int krylov_iterations;     /* interface iterations over all analyses       */
  double avg_krylov;         /* per analysis                                 */
  double compliance;         /* of the last analysis                          */
  double max_change, volume; /* of the last update                           */
  double t_total_ms, t_moduli_ms, t_solve_ms, t_update_ms;
} edd_topopt_stats;

/* Defaults: volfrac 0.5, rho in [1e-3, 1], move 0.2, eta 0.5, penal 1,
 * emin 0 (Variable Thickness Sheet), change_tol 1e-2, maxit 100, adaptive
 * tolerance in [1e-8, 1e-2], warm start. */
void edd_default_topopt_opts(edd_topopt_opts *o);

/* Run the loop from the densities in rho_dev (n_el values, overwritten by
 * the final design); u_dev (full nodal vector) receives the last analysis.
 * so: options of the analyses (tol and use_initial_guess are set by the
 * loop; NULL = edd_default_opts).  st may be NULL.  history_host (NULL or
 * 5 * maxit doubles) receives per step: compliance, Krylov tolerance,
 * interface iterations, max density change, final relative residual.
 * Synchronises. */
int edd_topopt_run(edd_problem *p, const double *f_dev, double *rho_dev, double *u_dev,
                   const edd_topopt_opts *to, const edd_solve_opts *so,
                   edd_topopt_stats *st, double *history_host);

/* ---- kernel timing ----------------------------------------------------- */
#define EDD_KT_BAND_SOLVE 0    /* batched forward+backward substitution,   */
                               /* FP64 factors                             */
#define EDD_KT_BAND_CHOLESKY 1 /* batched band Cholesky                    */
#define EDD_KT_APPLY_K 2       /* full matrix-free K apply                 */
#define EDD_KT_APPLY_MAPPED 3  /* K apply restricted to interior/interface */
#define EDD_KT_ASSEMBLE 4      /* band assembly of K_II                    */
#define EDD_KT_PRECOND 5       /* interface preconditioner kernels         */
#define EDD_KT_LAYOUTS 6       /* solve layouts of the interior factors    */
#define EDD_KT_BAND_SOLVE32 7  /* the substitutions with FP32 factors      */
#define EDD_KT_COUNT 8

typedef struct edd_kernel_times {
  int64_t count[EDD_KT_COUNT];   /* launches timed                          */
  double total_ms[EDD_KT_COUNT]; /* sum of their durations (HIP events on   */
                                 /* the handle's stream around each launch) */
} edd_kernel_times;

/* Enable (1) or disable (0) per-launch timing of the kernel families above
 * and reset the counters.  Timing adds two event records per launch. */
int edd_set_kernel_timing(edd_problem *p, int enable);

/* Resolve pending events (synchronises) and return the accumulated times. */
int edd_get_kernel_times(edd_problem *p, edd_kernel_times *t);

/* Release everything owned by the handle (NULL is accepted).  Synchronises. */
int edd_destroy(edd_problem *p);

/* Static description of a status code. */
const char *edd_strerror(int code);

/* The last hipError_t recorded on the handle (0 when none). */
int edd_last_hip_error(edd_problem *p);

#ifdef __cplusplus
}
#endif
#endif /* EDD_H */

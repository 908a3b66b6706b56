/*
 * ahoc.h -- C ABI of the MI355X (gfx950) augmented high-order-compact solver
 * for clamped, variable-coefficient biharmonic problems.
 *
 * Problem (Section 2, eq. (1) with the boundary conditions eq-bc):
 *     -Delta( alpha Delta u ) + beta Delta u = f   in the box [lo_0,hi_0] x ... (dim 2 or 3)
 *     u = g_D,  du/dn = g_N          on clamped faces (all faces by default)
 *     u = g_D,  Delta u = g_L        on Navier faces (ahoc_problem.navier)
 * with beta a constant (0 by default)
 * discretised by the fourth-order compact scheme of Sec. 2.2 (19-point L_h and
 * 7-point M in 3-D, 9-point L_h and 5-point M in 2-D) on a uniform grid with
 * n[a] intervals per axis.  The unknown boundary values Q of v = alpha Delta u
 * on the face interiors are found from the Schur-complement system S_h Q = b
 * (Sec. 2.3, eq-schur) with a matrix-free GMRES whose matrix-vector product is
 * Lemma 1 / Algorithm 1 (SchurMatVec): two DST-I fast Poisson solves, the
 * variable-coefficient weighting M(V/alpha), and the one-sided boundary
 * residual gather.
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer (HIP device memory) unless
 *     stated otherwise.  Nodal arrays hold (n_z+1)(n_y+1)(n_x+1) doubles
 *     (2-D: (n_y+1)(n_x+1)), x fastest.
 *   - Q (length ahoc_nq) is ordered by faces x-, x+, y-, y+[, z-, z+]; inside a
 *     face the two tangential axes are row-major, lower axis fastest.
 *   - The caller owns every buffer it passes.  ahoc_setup copies what it needs
 *     into handle-owned device memory, so problem arrays may be freed after
 *     setup returns.
 *   - `stream` is a hipStream_t (NULL = the default stream).  ahoc_setup,
 *     ahoc_solve and ahoc_solve_batched return after the work has completed;
 *     ahoc_schur_apply, ahoc_precond_apply, ahoc_schur_rhs, ahoc_poisson and ahoc_dst1
 *     are asynchronous on the stream.  No entry point synchronises the whole device:
 *     waits are on the call's stream, or (ahoc_destroy, ahoc_profile,
 *     ahoc_kernel_times) on events recorded after the handle's own work.
 *   - Device memory of a handle comes from the caller's ahoc_allocator when one is
 *     given (e.g. a framework's caching allocator), else from hipMalloc.
 *   - Errors are reported by return code only; ahoc_last_error() gives text.
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef AHOC_H
#define AHOC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AHOC_OK = 0,
  AHOC_E_INVALID = -1,     /* bad argument: dim, sizes, NULL arrays, alpha <= 0 */
  AHOC_E_NOMEM = -2,       /* device allocation failed                           */
  AHOC_E_NOCONV = -3,      /* tolerance not reached; outputs hold the last iterate */
  AHOC_E_HIP = -4,         /* a HIP runtime call failed                          */
  AHOC_E_UNSUPPORTED = -5  /* an option or problem combination the library does not solve
                              (see ahoc_problem, ahoc_options)                     */
} ahoc_status;

typedef enum {
  AHOC_FP64 = 0,  /* every step in FP64                                          */
  AHOC_MIXED = 1  /* FP32 transforms/stencils inside FP64 iterative refinement;
                     residual, Krylov vectors, Arnoldi, Givens, updates in FP64   */
} ahoc_precision;

/* One problem of eq. (1), -Delta(alpha Delta u) + beta Delta u = f, clamped on every face
 * unless `navier` marks it.  alpha and f are required; gD, gN, lapgD, gL may be NULL (= 0).
 *   alpha  nodal coefficient, must satisfy alpha > 0 everywhere (checked)
 *   f      nodal right-hand side in the sign of eq. (1)
 *   beta   a constant; 0 for the biharmonic-type problem.  beta != 0 needs a constant
 *          alpha (the v-equation -L_h V + (beta/alpha) M V = M f is then solved by the
 *          sine transforms with a shifted eigenvalue) and, in MIXED precision, the Schur
 *          refinement (refine = 1); otherwise AHOC_E_UNSUPPORTED
 *   gD     nodal; boundary entries are the Dirichlet data u = g_D
 *   gN     nodal; on face-interior nodes the OUTWARD normal derivative of u
 *   lapgD  nodal; on face-interior nodes the tangential part of Delta u fixed by
 *          g_D (Sec. 2.2 boundary Laplacian decomposition); on edges and corners
 *          the full Delta u (Remark 1)
 *   navier bit f (f = 2*axis + side, side 0 = low face; axes x, y[, z]) set: face f is a
 *          Navier face, u = g_D and Delta u = g_L there instead of du/dn = g_N (the
 *          boundary conditions eq-bc on the Navier part of the boundary).  Then v = alpha
 *          g_L is known on that face, and its rows of the Schur system read
 *          alpha g_L - Q = 0.  Bits beyond the 2*dim faces: AHOC_E_INVALID.
 *          ahoc_solve_batched batches 2-D problems of equal grids and equal Navier faces
 *          (beta = 0) together
 *   gL     nodal; on face-interior nodes of Navier faces the given Delta u (read there
 *          only)
 *   beta_nodal  nodal; when not NULL a variable beta (the constant `beta` is then
 *          ignored): the v-equation -L_h V + M(beta V / alpha) = M f is no longer diagonal
 *          in the sine basis and each V-solve runs BiCGSTAB preconditioned by the sine
 *          transform solve with the constant shift (min + max)/2 of beta/alpha (Remark 2).
 *          FP64 precision only (AHOC_MIXED: AHOC_E_UNSUPPORTED); set up alone */
typedef struct {
  int dim;       /* 2 or 3 */
  int n[3];      /* intervals per axis, 4 <= n[a] <= 8192 (unused axis ignored); the
                    one-sided normal formula of Sec. 2.2 reads U_1..U_3, so n[a] >= 4.
                    Lengths with radix-2/3 factors use the FFT passes, any other length
                    a direct sine-sum pass (O(n) work per output)                 */
  double lo[3];
  double hi[3];
  const double* alpha;
  const double* f;
  const double* gD;
  const double* gN;
  const double* lapgD;
  double beta;
  int navier;
  const double* gL;
  const double* beta_nodal;
  /* equation: AHOC_BIHARMONIC (0) for eq. (1) above, or AHOC_TRIHARMONIC (1) for the
   * sixth-order problem of Sec. 4.2, Delta^3 u = f (f in that sign; alpha, beta, lapgD, gL
   * and beta_nodal unused), solved as Delta u = v, Delta v = w, Delta w = f with the compact
   * scheme and w = Q on the face interiors.  Clamped faces carry u = g_D, u_n = g_N,
   * u_nn = gNN; Navier faces u = g_D, Delta u = lapu, Delta^2 u = bilap.  The q-row of a
   * clamped face is the augmented equation q = Delta^2 u with the one-sided fourth normal
   * derivative of U from U_1..U_4 and u, u_n, u_nn (so n[a] >= 5), plus tang4.  The
   * boundary-symbol preconditioner (precond = 1) takes the triharmonic chain's face-pair
   * symbol; MIXED needs refine = 1; v outputs and batches of lock-step instances are not
   * offered (AHOC_E_UNSUPPORTED for v, solo jobs in ahoc_solve_batched).  Arrays nodal,
   * NULL = 0:
   *   gNN    on face-interior nodes of clamped faces: the second normal derivative of u
   *   lapu   on every boundary node: Delta u (on a clamped face u_nn plus the tangential
   *          Laplacian of g_D)
   *   bilap  on Navier faces, edges and corners: Delta^2 u
   *   tang4  on face-interior nodes of clamped faces: Delta^2 u minus its pure normal part
   *          u_nnnn (what g_D and gNN fix) */
  int equation;
  const double* gNN;
  const double* lapu;
  const double* bilap;
  const double* tang4;
} ahoc_problem;

enum { AHOC_BIHARMONIC = 0, AHOC_TRIHARMONIC = 1 };

typedef struct {
  int precision;      /* ahoc_precision                                              */
  int restart;        /* GMRES restart length m (default 30)                         */
  int max_iters;      /* cap on GMRES iterations per Schur solve (default 2000)      */
  double tol;         /* relative Schur residual ||b - S Q|| / ||b|| (1e-12): the FP64
                         solve's GMRES tolerance, the MIXED (refine = 1) sweep stop    */
  double inner_tol;   /* MIXED: relative Schur residual of each correction (1e-5); the
                         inner solve also ends when FP32 rounding stalls its residual   */
  double sweep_tol;   /* MIXED, refine = 0: stop when the estimated remaining relative
                         change of U (max norm) is below this (default 1e-11)         */
  int max_sweeps;     /* MIXED: refinement sweeps cap (default 8)                    */
  int tile_fp64;      /* DST work-group tile in pencil pairs, 0 = default            */
  int tile_fp32;
  int precond;        /* 1 (default): right-precondition GMRES with the boundary symbol
                         (Sec. 4 solver settings; see ahoc_precond_apply); 0: none     */
  int refine;         /* MIXED refinement: 1 (default) on the Schur system -- FP64
                         residual b - S_h Q (FP64 operator), FP32-operator corrections,
                         stop when ||b - S_h Q|| <= tol ||b||, FP64 recovery of U, V;
                         0 on the coupled system -- FP64 residual of all three equation
                         groups, corrections solved and recovered in FP32, stop on
                         sweep_tol                                                     */
  int use_graph;      /* 1: the GMRES operator of each Krylov step (boundary-symbol
                         preconditioner and Schur matvec) is captured once as a HIP graph
                         and replayed; needs a stream that can be captured (not the
                         legacy default stream: there the launches stay eager).  Ignored
                         while ahoc_profile is on and with a variable beta (its V-solve
                         synchronises on dot products).  0 (default): eager launches   */
  int warm_start;     /* 1: the q argument of ahoc_solve holds an initial guess Q_0 on entry
                         (Sec. 4.1 starts GMRES from the interpolated coarse-grid solution);
                         GMRES (FP64) or the Schur refinement (MIXED, refine = 1) starts
                         from it, and the first residual b - S_h Q_0 costs one Schur matvec.
                         0 (default): Q_0 = 0 and q is output only.  MIXED with refine = 0:
                         AHOC_E_UNSUPPORTED.  Ignored by ahoc_solve_batched             */
  int vsolve_max_iters; /* variable beta: BiCGSTAB iteration cap of each V-solve (0 = 200) */
} ahoc_options;

typedef struct {
  int converged;
  int gmres_iters;       /* total over sweeps                           */
  int sweeps;            /* refinement sweeps (1 for FP64)              */
  int matvecs;           /* Schur matrix-vector products                */
  double schur_relres;   /* last GMRES relative residual estimate       */
  double last_update;    /* last sweep's max |dU| / max |U|             */
  double t_solve_ms;     /* wall time of ahoc_solve                     */
  int graph_steps;       /* Krylov steps whose operator ran as a HIP graph replay
                            (use_graph); 0 when the launches stayed eager  */
  int dst_gemm;          /* bit 2*axis + kind set where the operator of the solve's
                            precision (FP32 for AHOC_MIXED) runs that axis's plain
                            DST-I passes (kind 0 contiguous, 1 strided) as the
                            matrix-core pass (see ahoc_dst_choice)       */
  int vsolve_iters;      /* variable beta: BiCGSTAB iterations over all V-solves
                            (0 otherwise)                                  */
  double vsolve_relres;  /* variable beta: the largest final relative residual
                            ||r|| / ||rhs|| of any V-solve of the call (0 otherwise).
                            Above 1e-10 the Schur operator was applied inexactly and the
                            call returns AHOC_E_NOCONV with converged = 0  */
} ahoc_stats;

/* Device memory provider.  alloc returns `bytes` bytes of device memory of the current
 * device, at least 256-byte aligned, or NULL on failure (then the call returns
 * AHOC_E_NOMEM); free releases a pointer alloc returned.  The library frees only memory
 * whose work has completed (ahoc_destroy waits for the handle's last work first).  The
 * callbacks may run concurrently on the worker threads of ahoc_solve_batched and must be
 * thread-safe.  ctx is passed through unchanged. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} ahoc_allocator;

typedef struct ahoc_handle ahoc_handle;

/* Fill `opt` with the defaults listed above. */
void ahoc_default_options(ahoc_options* opt);

/* Validate the problem, derive 1/alpha, M f, the boundary data lifts and the
 * transform tables, allocate the workspace (through `alloc`, or hipMalloc when it is
 * NULL; the handle keeps the allocator and releases through it).  Returns
 * AHOC_E_INVALID for dim not in {2,3}, n[a] outside [4, 8192], hi <= lo, NULL alpha/f or
 * min alpha <= 0, AHOC_E_NOMEM when an allocation fails, AHOC_E_UNSUPPORTED for an
 * option/problem combination listed as such.  *out is set only on success; release it
 * with ahoc_destroy. */
ahoc_status ahoc_setup(const ahoc_problem* prob, const ahoc_options* opt, const ahoc_allocator* alloc,
                       void* stream, ahoc_handle** out);

/* Number of augmented unknowns N_q of the handle's grid. */
size_t ahoc_nq(const ahoc_handle* h);

/* y = S_h q (Lemma 1 in homogeneous form: R(q) - R(0)), q and y of length N_q,
 * FP64 in and out; the transforms and stencils run in the handle's precision. */
ahoc_status ahoc_schur_apply(ahoc_handle* h, const double* q, double* y, void* stream);

/* y = P^{-1} q for the boundary-symbol preconditioner of the handle (Sec. 4 names a
 * boundary-symbol preconditioner for the Schur GMRES without defining it).  P is the
 * Schur complement of the constant-coefficient (alpha = 1) problem restricted to each
 * pair of opposite faces: diagonal in the faces' 2-D sine basis up to the 2x2 coupling of
 * the two faces, inverted mode by mode.  q, y: length N_q, FP64; asynchronous on the
 * stream; AHOC_E_INVALID if the handle was set up with precond = 0. */
ahoc_status ahoc_precond_apply(ahoc_handle* h, const double* q, double* y, void* stream);

/* Right-hand side b = -R(0) of the Schur system (Algorithm 1, ConstructSchurRHS), FP64, length N_q.
 * It is the right-hand side the handle's solve uses: formed with the FP64 operator, except
 * for MIXED with refine = 0, whose first sweep forms it with the FP32 operator. */
ahoc_status ahoc_schur_rhs(ahoc_handle* h, double* b, void* stream);

/* Solve.  u (nodal, required) receives U; v (nodal or NULL) receives V = alpha Delta u
 * (interior V, Q on face interiors, alpha*lapgD on edges/corners); q (length N_q or
 * NULL) receives Q (and holds the initial guess on entry with options.warm_start = 1).
 * stats may be NULL.  Returns AHOC_E_NOCONV when the tolerance is not met -- the
 * iteration cap, an FP32 stall, or a non-finite right-hand side or residual (NaN or Inf
 * in the data) -- with converged = 0 and the outputs holding the last iterate: Q as
 * GMRES left it and U, V recovered from that Q. */
ahoc_status ahoc_solve(ahoc_handle* h, double* u, double* v, double* q, ahoc_stats* stats,
                       void* stream);

/* Solve `count` independent problems (sizes and coefficients may differ) with
 * shared options and allocator (NULL = hipMalloc).  u is a HOST array of `count` device
 * pointers; stats a host array of `count` entries (or NULL).  Returns the first non-OK
 * status. */
ahoc_status ahoc_solve_batched(int count, const ahoc_problem* probs, const ahoc_options* opt,
                               const ahoc_allocator* alloc, double* const* u, ahoc_stats* stats,
                               void* stream);

/* Dirichlet solve with the compact operator on the handle's interior grid:
 * w = L_int^{-1} g (homogeneous boundary), g and w interior arrays of FP64
 * ((n_z-1)(n_y-1)(n_x-1), x fastest), in the handle's precision internally. */
ahoc_status ahoc_poisson(ahoc_handle* h, const double* g, double* w, void* stream);

/* For callers that cannot allocate device memory -- code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc -- the Dirichlet solve of ahoc_poisson
 * without a handle: w = L_int^{-1} g on the interior of a dim-D box grid with n[a]
 * intervals (4 <= n[a] <= 8192) and spacings (hi[a] - lo[a]) / n[a], homogeneous boundary;
 * g and w interior FP64 arrays ((n_z-1)(n_y-1)(n_x-1), x fastest, no padding; w may equal g),
 * computed in FP64 (AHOC_FP64) or with FP32 transforms (AHOC_MIXED).  The work array and
 * the transform tables live in one fixed device array of 64 MiB per GPU, held by the
 * library until the process ends (1 MiB of tables, then the interior padded to rows of a
 * multiple of 32 elements): a grid whose padded interior exceeds 63 MiB in the working
 * precision returns AHOC_E_INVALID.  Allocates nothing (no hipMalloc, hipFree or allocating
 * library call) and copies nothing from the host; asynchronous on the stream.  Every call on
 * a GPU shares that GPU's array and leaves its contents behind: calls that overlap on one GPU
 * (other streams, other threads) race and must be serialised by the caller. */
ahoc_status ahoc_poisson_noalloc(int precision, int dim, const int* n, const double* lo, const double* hi,
                                 const double* g, double* w, void* stream);

/* Stand-alone batched DST-I along one axis of an interior-shaped array:
 * out[..., k, ...] = sum_{m=1}^{N-1} in[..., m, ...] sin(pi k m / N), N = nint[axis]+1.
 * precision: AHOC_FP64 (double arrays) or AHOC_MIXED (float arrays).
 * nint: interior sizes (x, y[, z]); in may equal out. */
ahoc_status ahoc_dst1(int precision, int dim, const int* nint, int axis, const void* in, void* out,
                      void* stream);

/* Select the DST-I pass kernel family for subsequent launches (process-wide):
 * 0 = automatic (length-specialised kernels for n in {32, 64, 96, 128, 192, 256, 384,
 * 512, 768, 1024, 2048, 4096}, the generic radix-2/3/4/8 kernel otherwise; for the plain
 * passes of an operator the kernel ahoc_setup's timing chose, see ahoc_dst_choice),
 * 1 = generic kernel for every length, 2 = specialised kernels only (other lengths
 * return AHOC_E_UNSUPPORTED), 3 = as 0 but strided passes with the one-tile-per-group
 * kernels instead of the persistent pipelined ones, 4 = the matrix-core products for every
 * plain pass of even n <= 128 (untimed), 5 = as 0 without setup-time choices (default
 * kernels).
 * Handles keep the choice timed at their setup.  For tuning and for testing every
 * family: a process-wide switch read by every pass launched after the call (atomically;
 * passes that other threads launch while it changes may run either family), not a
 * per-handle setting.  Production callers leave it at 0. */
ahoc_status ahoc_set_dst_variant(int variant);

/* Calibration copies (no arithmetic): out = in for an [nz][ny][nx] FP32 volume, with the
 * global access pattern of pattern 0 = a linear copy (16-byte accesses), 1 = the strided DST
 * passes along y (persistent work-groups of 1024 threads, tiles of 32 columns = 128-byte row
 * segments across the ny rows of a plane), 2 = the strided passes along z (the same tiles
 * across the nz planes).  They measure the bandwidth the passes' access patterns allow on
 * the device (the roofline the DST kernels are compared with).  in, out: device pointers to
 * nx*ny*nz floats, owned by the caller (in == out allowed); nx must be a multiple of 32.
 * Asynchronous on the stream.  AHOC_E_INVALID on a bad argument. */
ahoc_status ahoc_copy_bandwidth(int pattern, const float* in, float* out, int nx, int ny, int nz, void* stream);

/* The setup-time choice of kernel for the plain DST-I passes along one axis of the
 * operator (the sine transforms of Sec. 2.3; every candidate gives the same transform up to
 * rounding).  ahoc_setup times, on the handle's own pass shape and in automatic kernel
 * selection only, the default FFT kernel (row kernel, or persistent pipelined strided
 * kernel), the one-tile FFT kernel with half, the default and twice the default pencil pairs
 * per work-group (for n = 512, 1024 also a 32-point-per-thread radix plan), and for even
 * n <= 128 the matrix-core pass (two half-size sine-matrix products: odd outputs from
 * x_m + x_{n-m}, even ones from x_m - x_{n-m}), and keeps the fastest.  The first timing of
 * a shape (precision, n, pass extents) is kept for the process, so later handles with the
 * same shape make the same choice and give bit-identical results.
 * precision: AHOC_FP64 (the FP64 operator) or AHOC_MIXED (the FP32 operator);
 * kind: 0 = contiguous (x) passes, 1 = strided passes (y, 3-D only).
 * Out: *method = 0 default FFT kernel, 1 matrix-core pass, 2 one-tile FFT kernel with *tile
 * pencil pairs per work-group, -1 not timed (a pass kind the operator does not run on this
 * axis, or a non-automatic variant); *tile = pairs for method 2, else 0; *t_default_us,
 * *t_gemm_us, *t_best_us = measured microseconds per pass of the default kernel, the
 * matrix-core pass and the chosen kernel, -1 when not timed or not applicable.  Each
 * pointer but method may be NULL.  AHOC_E_INVALID on a bad argument, AHOC_E_UNSUPPORTED
 * when the handle has no operator in that precision. */
ahoc_status ahoc_dst_choice(const struct ahoc_handle* h, int precision, int axis, int kind, int* method, int* tile,
                            double* t_default_us, double* t_gemm_us, double* t_best_us);

/* Override the default work-group tile (pencil pairs per work-group, a power of two;
 * 0 restores the default) of one DST-I pass kind of the length-specialised kernels,
 * process-wide: pass 0 = rows (contiguous pencils), 1 = strided pencils, 2 = fused
 * forward/scale/inverse pass; precision selects the FP64 or the FP32 (AHOC_MIXED)
 * kernels.  A tile whose work-group exceeds the kernel's size or LDS limits makes the
 * launch return AHOC_E_UNSUPPORTED; the fused pass clamps it to its default.  The
 * per-handle ahoc_options.tile_* fields take precedence.  For tuning: process-wide and
 * read atomically by every pass launched after the call, as ahoc_set_dst_variant. */
ahoc_status ahoc_set_dst_tile(int pass, int precision, int pairs);

/* Kernel classes for ahoc_kernel_times. */
enum {
  AHOC_K_DST_ROWS = 0,     /* DST-I pass along x (contiguous pencils)                   */
  AHOC_K_DST_STRIDED = 1,  /* DST-I pass along y in 3-D (strided pencils)               */
  AHOC_K_DST_FUSED = 2,    /* fused forward DST and eigen scaling along the slowest axis, then
                              the inverse DST (Poisson solves) or the face sums (U-solve)  */
  AHOC_K_LIFT = 3,         /* v-equation right-hand side from Q (face layers and their
                              2-D spectra in the spectral form)                           */
  AHOC_K_RHS_U = 4,        /* u-equation right-hand side M(V/alpha)                      */
  AHOC_K_GATHER = 5,       /* boundary residual gather (with the face-sum reductions and
                              2-D inverse transforms in the spectral form)                */
  AHOC_K_KRYLOV = 6,       /* one Arnoldi step (CGS2 dots/axpys, norm, Givens, scale)     */
  AHOC_K_RESID = 7,        /* FP64 coupled residual (mixed precision)                    */
  AHOC_K_MATVEC = 8,       /* one whole Schur matrix-vector product                      */
  AHOC_K_DST_GEN = 9,      /* V-solve: spectrum of the face-layer lift generated, scaled and
                              inverted along the slowest axis (writes the volume only)     */
  AHOC_K_FACE_REDUCE = 10, /* U-solve: face sums along the two fastest axes from the stored
                              scaled spectrum (reads the volume only)                      */
  AHOC_K_PRECOND = 11,     /* one application of the boundary-symbol preconditioner       */
  AHOC_K_VSOLVE = 12,      /* variable beta: one BiCGSTAB V-solve with its transform solves
                              and stencil applications (bytes not modelled)               */
  AHOC_K_DST_XMUL = 13,    /* 3-D matvec: the V-solve's inverse and the U-solve's forward
                              DST-I along x with the product by 1/alpha between them      */
  AHOC_NKIND = 14
};

/* Enable (1) or disable (0) per-kernel-class timing of the handle's solves with
 * HIP events recorded on the solve stream around each launch; resets the totals (waits
 * for the handle's pending timing events, not for the device). */
ahoc_status ahoc_profile(ahoc_handle* h, int enable);

/* Accumulated time (ms) and launch count of one kernel class since ahoc_profile,
 * and the algorithmic bytes one launch moves on average (what the operation must
 * read and write at least once).  Waits for the handle's pending timing events.  Any
 * output may be NULL. */
ahoc_status ahoc_kernel_times(ahoc_handle* h, int kind, double* total_ms, long long* launches,
                              double* bytes_per_launch);

/* Release a handle: waits for the work it enqueued (an event recorded after its last
 * call, not a device-wide synchronisation), then frees its memory through its allocator. */
void ahoc_destroy(ahoc_handle* h);

const char* ahoc_status_string(ahoc_status s);
/* Text of the last error recorded by this library (thread-local). */
const char* ahoc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AHOC_H */

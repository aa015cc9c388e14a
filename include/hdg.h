/*
 * hdg.h -- C ABI of the MI355X (gfx950) unified geometric multigrid solver
 * for the statically condensed HDG trace system.
 *
 * The method: hybridized DG discretization of -div(kappa grad u) = f with
 * Dirichlet data (Sec. 2, eqs. primal_elliptic, mixed_elliptic, HDG,
 * HDG_flux), static condensation to the trace system A lambda = g
 * (eq. trace_linear_system), and the multigrid of Sec. 3: p-coarsening to
 * P1 (Sec. 3.1.1), h-coarsening by agglomeration (eq. trace_partition),
 * DtN-based prolongation/restriction (eqs. n_1_Ik, n_g1_Ik, n_1_Qk,
 * n_g1_Qk), Galerkin coarse operators (eqs. Akm1, ANm1), face-block Jacobi
 * smoothing (Sec. 3.3, Sec. 4.1), local correction (eq. localCorrection),
 * the V-cycle (Algorithm 1) used as a solver (Sec. 3.6) or as a CG/GMRES
 * preconditioner (Sec. 4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Mesh: the unit box [0,1]^d, d in {2,3}, n^d equal quads/hexes, h = 1/n.
 *   Elements are numbered lexicographically, x fastest.
 * Spaces: Q^k on elements, nodal at tensor Gauss-Lobatto-Legendre points
 *   (x fastest); Q^k on faces (P^k in 2D) nodal at GLL points ordered by
 *   increasing global coordinate, first tangential direction fastest.
 * Trace vectors (lambda, g, residuals): interior faces only, face-major.
 *   x-normal faces first, then y (then z); within a direction the faces
 *   are lexicographic on the grid of extent n-1 along the normal and n
 *   elsewhere (x fastest); (k+1)^(d-1) values per face.
 * Boundary trace data: block (c, side) for c = 0..d-1, side = 0 (x_c=0),
 *   1 (x_c=1); inside a block the n^(d-1) faces are lexicographic over the
 *   tangential coordinates; (k+1)^(d-1) values per face.
 * Volume arrays: u[N_T][(k+1)^d], q[N_T][d][(k+1)^d], nodal.
 * Source: nodal values f[N_T][(k+1)^d] (its interpolant is integrated
 *   exactly: load b_T = M_T f_T), or a load vector in the same layout.
 * kappa: per element [N_T] (HDG_KAPPA_PER_ELEMENT) or at the tensor Gauss
 *   points with k+2 points per direction [N_T][(k+2)^d] (HDG_KAPPA_AT_QP).
 *
 * Memory: every array argument is a DEVICE pointer owned by the caller,
 * except the option/info structs, which live on the host.  The library
 * copies what it keeps and never frees caller memory.  The handle owns all
 * internal device memory (allocated in setup/build, freed in destroy).
 * Work is ordered on the stream given at setup; calls that fill an info
 * struct synchronize that stream.  A handle is not thread-safe; distinct
 * handles are independent.  Every call returns an hdg_status; nothing
 * throws across the ABI.  On HDG_ERR_NOT_CONVERGED the output holds the
 * last iterate and info is filled.
 */
#ifndef HDG_H
#define HDG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hdg_problem* hdg_handle;

typedef enum {
  HDG_OK = 0,
  HDG_ERR_INVALID_ARG = -1,   /* null pointer, bad size, kappa <= 0 or not finite, ... */
  HDG_ERR_UNSUPPORTED = -2,   /* e.g. n not a power of two at mg_build, k or d out of range */
  HDG_ERR_STATE = -3,         /* e.g. solve before mg_build */
  HDG_ERR_NOT_CONVERGED = -4, /* max_it reached; outputs hold the last iterate */
  HDG_ERR_BREAKDOWN = -5,     /* non-finite residual or zero Krylov denominator */
  HDG_ERR_DEVICE = -6         /* a HIP call failed */
} hdg_status;

enum { HDG_KAPPA_PER_ELEMENT = 0, HDG_KAPPA_AT_QP = 1 };
enum { HDG_FP64 = 0, HDG_FP32 = 1, HDG_MIXED = 1, HDG_MIXED_CYCLE = 2 /* hdg_vcycle only, see there */ };
enum { HDG_LC_NONE = 0, HDG_LC_PRE = 1, HDG_LC_POST = 2, HDG_LC_BOTH = 3 };
enum { HDG_METHOD_MG = 0, HDG_METHOD_PCG = 1, HDG_METHOD_GMRES = 2 };
enum { HDG_RHS_F_NODAL = 0, HDG_RHS_F_LOAD = 1, HDG_RHS_TRACE = 2 };
#define HDG_MAX_NRHS 64 /* right-hand sides one group of a solve or V-cycle can hold */

typedef struct {
  int dim;          /* 2 or 3 */
  int n;            /* elements per direction; a power of two for mg_build */
} hdg_mesh;

typedef struct {
  int sweeps;       /* block-Jacobi sweeps before and after the coarse correction on the finest level (default 2) */
  int growth;       /* 1: same sweeps on every level; 2: doubled per coarser level (Sec. 3.3, beta0 = beta1 = 2) */
  double omega;     /* block-Jacobi damping (default 1, Sec. 4.1) */
  int local_corr;   /* HDG_LC_*: Algorithm 1 step 3 (PRE), step 5 (POST) or both */
  int precision;    /* HDG_FP64 or HDG_MIXED (FP32 V-cycle inside FP64 outer iteration) */
  int method;       /* HDG_METHOD_MG | PCG | GMRES (GMRES: right preconditioned, MGS) */
  int max_it;       /* outer iteration limit (default 200, Sec. 4) */
  int restart;      /* GMRES restart length (0: no restart up to max_it) */
  int coarse_n;     /* stop h-coarsening at the first macro grid with <= coarse_n macro-elements per
                       direction and solve it directly (B_1 = A_1^-1); 2 (default) coarsens to 2 x 2.
                       The paper leaves the number of levels free (Sec. 3.1.2, Sec. 4.5). */
  int nrhs;         /* right-hand sides one solve or V-cycle call iterates together (1 .. HDG_MAX_NRHS);
                       larger counts go through in groups of this size.  Every kernel of the cycle and
                       of CG then runs all of them in one launch, and the trace apply reads each
                       operator block once for the group (through the L2 of its XCD). */
  double refine_red;/* HDG_MIXED with PCG: each FP64 refinement step runs the FP32-preconditioned CG
                       until its residual has dropped by this factor against the step's true FP64
                       residual (or stagnates), then recomputes g - A lambda in FP64 and restarts
                       (0: default 1e-5).  Unused in FP64. */
  int variant;      /* HDG_VARIANT_* bits: select another execution form of the same method (for
                       comparing forms; 0 = the default, fastest form).  Iterates agree up to the
                       order of rounding. */
  int smoother;     /* HDG_SMOOTHER_* (Sec. 4.1): face-block Jacobi (default) or a point smoother.  The
                       point smoothers store every level face-major and use the unfused kernels. */
} hdg_mg_opts;

/* Smoothers of Sec. 4.1.  JACOBI: damped point Jacobi, x += omega D^-1 (b - A x) (the paper takes
   omega = 2/3).  CHEBYSHEV: point Jacobi accelerated by the Chebyshev polynomial of degree m (the
   level's sweep count) on [lmax / 30, lmax], lmax = 1.1 x a power-iteration estimate of the largest
   eigenvalue of D^-1 A (20 steps from the all-ones vector), applied as m Jacobi steps with step sizes
   the reciprocals of the polynomial's roots.  LUSGS: one forward and one backward point Gauss-Seidel
   sweep per step, in a multicolour order: faces in 2d colours no two of which share an element, the
   values within a face one after another (the paper sweeps in the plain unknown order, which has no
   parallel form). */
enum { HDG_SMOOTHER_BLOCK_JACOBI = 0, HDG_SMOOTHER_JACOBI = 1, HDG_SMOOTHER_CHEBYSHEV = 2, HDG_SMOOTHER_LUSGS = 3 };

/* Execution-form bits of hdg_mg_opts.variant. */
enum {
  HDG_VARIANT_NO_GRAPH = 1, /* launch iteration bodies eagerly instead of replaying captured HIP graphs */
  HDG_VARIANT_NO_FUSE = 2,  /* unfused level-transition kernels (residual, restriction, prolongation apart) */
  HDG_VARIANT_NO_TAIL = 4,  /* no one-workgroup coarse tail: every level launched on its own */
  HDG_VARIANT_NO_PACK = 8,  /* finest p-level stored face-major instead of element-major packed triangles */
  HDG_VARIANT_NO_STRIP = 16, /* element-major finest level applied in two passes instead of one strip pass */
  /* HDG_MIXED cycle form.  Default: in 3D every level keeps FP64 vectors and sums over the FP32 copies
     of its operator blocks (an FP32 cycle stalls CG near 1e-6 there); in 2D the whole cycle runs on FP32
     vectors.  These bits force one form (for comparing them); the FP64-vector form stores every level
     face-major and uses the unfused transition kernels. */
  HDG_VARIANT_FP32_VECTORS = 32, /* FP32 vectors and sums in the mixed cycle, also in 3D */
  HDG_VARIANT_FP64_VECTORS = 64, /* FP64 vectors and sums over FP32 operator blocks, also in 2D */
  /* Lanes per macro-element of the fused 2D h-transition kernels.  Default: four while macro-elements
     times right-hand sides stay below 16,384 (latency-bound levels), one above. */
  HDG_VARIANT_LANES1 = 128,     /* one lane per macro-element on every level */
  HDG_VARIANT_LANES4 = 256,     /* four lanes per macro-element (one interior face each) on every level */
  /* Coarse part of the 2D fused cycle (the h-levels from 128 x 128 down, and a coarsest level of more than
     64 unknowns) as one persistent launch, one workgroup per compute unit, phases separated by grid-wide
     barriers, single right-hand side; the same work items as the per-level kernels (results equal bit
     for bit).  The grid holds half as many workgroups as the device has compute units, so that all
     are resident together; a barrier wait that runs out of polls ends the solve with HDG_ERR_DEVICE.
     Batched solves refuse handles built with it.  Currently switched off (hdg_mg_build returns
     HDG_ERR_UNSUPPORTED for this bit): single V-cycles matched the per-level form bit for bit, but a
     graph-captured CG solve with it failed on the device for a reason not yet found. */
  HDG_VARIANT_GRID_TAIL = 512
};

typedef struct {
  int iters;        /* iterations of the outer method (V-cycles applied; for mixed PCG, CG steps over
                       all refinement steps) */
  double relres;    /* final ||g - A lambda||_2 / ||g||_2 computed in FP64 */
  double t_solve_ms;/* stream time of the solve */
  int n_levels;
  int outer_iters;  /* true FP64 residuals formed: refinement steps of mixed PCG, (re)starts otherwise */
  double t_setup_ms;/* host wall time of the handle's last hdg_setup / hdg_update_kappa (element maps) */
  double t_build_ms;/* host wall time of the handle's last hdg_mg_build (hierarchy) */
} hdg_solve_info;

/* Fill opts with the defaults above (constant 2 sweeps, omega 1, step-3
 * local correction, FP64, MG, 200 iterations, coarsening down to 2 x 2,
 * one right-hand side per group). */
void hdg_default_opts(hdg_mg_opts* opts);

/* Form the element-local HDG problems and their DtN matrices
 * A^e = tau H - S^T L^-1 R (static condensation, Sec. 2) on the device.
 * k in 1..6 for d = 2, 1..3 for d = 3; tau > 0.  kappa: device array laid
 * out per kappa_kind.  hip_stream: a hipStream_t (NULL = default stream).
 * store_recovery != 0 keeps the per-element factors needed by
 * hdg_reconstruct and hdg_adjoint.  On success *out owns the problem. */
hdg_status hdg_setup(const hdg_mesh* mesh, int k, double tau, const double* kappa, int kappa_kind,
                     int store_recovery, void* hip_stream, hdg_handle* out);

/* Discretizations of the trace system (Sec. 2): HDG (eqs. HDG, HDG_flux),
 * the hybridized interior penalty family of eq. IPG_H, with s_f = 1
 * (SIPG-H, eq. SIPG_H), 0 (IIPG-H) and -1 (NIPG-H), and the hybridized
 * Raviart-Thomas mixed method (RT-H, eqs. mixed_local1/2: RT_k =
 * Q_{k+1,k} x Q_{k,k+1} on the squares, scalar Q^k, traces P^k; d = 2,
 * k <= 4, no stabilization: tau is not used). */
enum { HDG_SCHEME_HDG = 0, HDG_SCHEME_SIPG = 1, HDG_SCHEME_IIPG = 2, HDG_SCHEME_NIPG = 3, HDG_SCHEME_RT = 4 };
/* Or-ed into the scheme of hdg_setup_scheme: element T is stabilized with
 * tau * kappa_T instead of tau (the paper's tau = kappa / h_min for HDG and
 * kappa (p+1)(p+2) / h_min for IPDG in Examples III and IV); needs
 * HDG_KAPPA_PER_ELEMENT, and hdg_adjoint does not take it. */
enum { HDG_SCHEME_TAU_KAPPA = 16 };

/* hdg_setup for any scheme.  For the IPDG schemes the element maps are
 *   A^e = tau H - C_T L_T^-1 R_T,  L_T = kappa (K - s_f N - N^T) + tau E,
 *   R_T = tau G - s_f kappa D,      C_T = tau G^T - kappa D^T
 * (eqs. IPDG_flux, IPG_H with the conservation rows of eq. conservation;
 * K the stiffness matrix, N_ij = <phi_j, grad phi_i . n>,
 * D_il = <mu_l, grad phi_i . n>, E, G, H the boundary mass matrices), the
 * load map is C_T L_T^-1 M_T, and recovery gives u_T and q_T = -kappa
 * grad u_T at the nodes.  IPDG takes kappa per element only
 * (HDG_KAPPA_AT_QP: HDG_ERR_UNSUPPORTED) and needs L_T to be nonsingular
 * with nonzero leading minors, which holds when its symmetric part is
 * positive definite (tau = (p+1)(p+2)/h_min does this for every s_f).
 * IIPG-H and NIPG-H give a nonsymmetric trace system: their builds reject
 * HDG_METHOD_PCG (HDG_ERR_UNSUPPORTED) and restrict with
 * Q = [-J^T A_BI A_II^-1, J^T] (eq. n_1_Qk) instead of I^T; hdg_adjoint
 * is HDG only.  Other arguments as for hdg_setup. */
hdg_status hdg_setup_scheme(const hdg_mesh* mesh, int k, double tau, const double* kappa, int kappa_kind,
                            int scheme, int store_recovery, void* hip_stream, hdg_handle* out);
/* (scheme: one HDG_SCHEME_* value, optionally | HDG_SCHEME_TAU_KAPPA.  For
 * RT-H the element maps are A^e = F^T Lqq F from the inverse of the local
 * saddle-point matrix [[M_q, -B], [B^T, 0]] (F the normal traces of the
 * velocity basis, M_q its kappa^-1 weighted mass, B_ij = (w_j, div v_i)),
 * the load map F^T Lqu M_T, and recovery returns u and the velocity field
 * evaluated at the scalar's nodes.) */

/* Multinumerics (Sec. 4.6): one discretization per element on a 2D mesh.
 * scheme_of_element: DEVICE array [N_T] of HDG_SCHEME_SIPG, _IIPG, _NIPG
 * or _RT (the trace spaces of these agree, so their element maps assemble
 * into one trace system; HDG elements are not mixed in); it is copied at
 * setup.  options: 0 or HDG_SCHEME_TAU_KAPPA (for the IPDG elements).
 * kappa per element when any IPDG element is present.  The operator is
 * symmetric when only SIPG-H and RT-H elements are present; otherwise the
 * build rules of the nonsymmetric schemes apply (no CG).  Recovery: u, and
 * the flux at the nodes (-kappa grad u on IPDG elements, the RT field on
 * RT-H elements).  Errors: HDG_ERR_INVALID_ARG for an unknown code,
 * HDG_ERR_UNSUPPORTED for d != 2, k > 4 with RT-H elements, or kappa at the
 * quadrature points with IPDG elements.  Other arguments as for hdg_setup. */
hdg_status hdg_setup_multi(const hdg_mesh* mesh, int k, double tau, const double* kappa, int kappa_kind,
                           const int* scheme_of_element, int options, int store_recovery, void* hip_stream,
                           hdg_handle* out);

/* Unstructured triangle meshes (Sec. 3.1.2 and Example II).  HOST arrays:
 * xy [nvert][2] vertex coordinates, tri [ntri][3] vertex indices listed
 * counter-clockwise, seeds [nseeds][2] the seed points of the level-1
 * macro-elements; hlevels agglomeration levels. */
typedef struct {
  long nvert;
  const double* xy;
  long ntri;
  const int* tri;
  int nseeds;
  const double* seeds;
  int hlevels;
} hdg_umesh;

/* HDG (eqs. HDG, HDG_flux; scheme HDG_SCHEME_HDG) or the hybridized IPDG
 * family (eq. IPG_H; HDG_SCHEME_SIPG, _IIPG, _NIPG, with the element blocks
 * of hdg_setup_scheme and recovery q = -kappa grad u) with P^k volume and
 * trace spaces on the triangles of an unstructured mesh, k in 1..4, scalar
 * tau > 0, kappa a DEVICE array with one value per triangle.  IIPG-H and
 * NIPG-H give a nonsymmetric trace system: CG is rejected and the
 * agglomeration levels restrict with -J^T A_BI A_II^-1 (eq. n_1_Qk).  Volume unknowns are nodal at
 * the equispaced lattice of each triangle (vertex 0 first, then along edge
 * 0; rows from edge 0 to vertex 2); the trace unknowns of an interior edge
 * are nodal at the GLL points of its parameter, which runs from its lower-
 * numbered vertex to the other; interior edges are numbered in order of
 * their sorted vertex pair; edges on the boundary carry zero Dirichlet data.
 * The multigrid hierarchy is fixed here (Sec. 3.1.2): level 1 gathers the
 * triangles nearest to each seed (centroid distance, lowest seed on ties;
 * seeds that win none are dropped), and each further level splits every
 * macro-element in four (halving twice at the median centroid along the
 * axis of larger centroid extent).  Macro-edges are the maximal chains of
 * finer faces shared by the same two macro-elements; their P^1 coarse
 * space is linear in arc length along the chain.  Levels: P^k on the
 * triangles, P^1 on the triangles (k > 1), then the agglomeration levels,
 * finest first; the coarsest is solved by a dense inverse (at most 4096
 * unknowns).  hdg_mg_opts.coarse_n > 2 stops the hierarchy at the coarsest
 * level with at least coarse_n^2 trace unknowns (the levels below are left
 * out and that level is solved directly); coarse_n <= 2 keeps every level.  hdg_mg_build takes block-Jacobi smoothing only (the mixed
 * precision cycle keeps FP64 vectors over FP32 operator blocks); hdg_rhs,
 * hdg_solve and hdg_reconstruct take nodal f (HDG_RHS_F_NODAL, [ntri][nv]
 * at the lattice nodes) and optional Dirichlet traces g_dirichlet
 * [nbedge][k+1] (boundary edges in order of their sorted vertex pair, GLL
 * values along each edge's parameter; NULL: zero); hdg_reconstruct returns
 * u [ntri][nv] and q [ntri][2][nv] at the lattice nodes.  The adjoint,
 * kappa updates, batches and the autotuner return HDG_ERR_UNSUPPORTED.  Errors: HDG_ERR_INVALID_ARG for clockwise or
 * degenerate triangles, edges shared by more than two triangles, or a
 * macro-element with more than 1024 trace values; HDG_ERR_UNSUPPORTED for
 * k outside 1..4. */
hdg_status hdg_setup_unstructured(const hdg_umesh* mesh, int k, double tau, const double* kappa, int scheme,
                                  void* hip_stream, hdg_handle* out);

/* Host only (no GPU call): the trace unknowns of every level of the
 * hierarchy hdg_setup_unstructured builds for this mesh and degree, finest
 * first, into sizes[0 .. *nlevels - 1] (for choosing coarse_n).  Errors as
 * for hdg_setup_unstructured; HDG_ERR_INVALID_ARG also when the hierarchy
 * has more than max_levels levels (*nlevels then holds the count). */
hdg_status hdg_umesh_levels(const hdg_umesh* mesh, int k, long long* sizes, int max_levels, int* nlevels);

/* Re-form A^e for a new kappa (same layout rules); invalidates the
 * hierarchy (call hdg_mg_build again). */
hdg_status hdg_update_kappa(hdg_handle h, const double* kappa, int kappa_kind);

/* Build the multigrid hierarchy of Sec. 3: J_N^T A J_N (eq. ANm1) for
 * k > 1, then per h-level the macro-element Schur complements
 * A_{k-1} = J^T (A_BB - A_BI A_II^-1 A_IB) J (eq. Akm1) with the local
 * factors A_II^-1 and P = -A_II^-1 A_IB J, face-block inverses, and the
 * coarsest dense inverse (B_1 = A_1^-1).  Needs n = 2^m, n >= 2. */
hdg_status hdg_mg_build(hdg_handle h, const hdg_mg_opts* opts);

/* One V-cycle e = B_L r on the finest level (Algorithm 1), r and e trace
 * vectors of length N_lambda (double for HDG_FP64, float for HDG_FP32, and
 * double for HDG_MIXED_CYCLE: the cycle the mixed solve applies, in the
 * build's mixed form); nrhs vectors stored one after another. */
hdg_status hdg_vcycle(hdg_handle h, const void* r, void* e, int precision, int nrhs);

/* Right-hand side g of eq. trace_linear_system from a volume source
 * (rhs_kind F_NODAL or F_LOAD, [N_T][(k+1)^d]) and optional Dirichlet
 * boundary traces g_dirichlet (boundary layout, NULL = 0); g: [N_lambda]. */
hdg_status hdg_rhs(hdg_handle h, const double* rhs, int rhs_kind, const double* g_dirichlet, double* g);

/* Solve A lambda = g to ||g - A lambda||_2 <= tol ||g||_2 with the method of
 * the build options.  rhs: volume source (F_NODAL/F_LOAD) or g itself
 * (TRACE).  lambda: in = initial guess, out = solution, [nrhs][N_lambda]. */
hdg_status hdg_solve(hdg_handle h, const double* rhs, int rhs_kind, const double* g_dirichlet, int nrhs,
                     double tol, double* lambda, hdg_solve_info* info);

/* Batched solves (many meshes, many right-hand sides): problem i solves its
 * nrhs[i] right-hand sides rhs[i] (layout as in hdg_solve) into lambda[i]
 * (in: initial guesses) with its own built handle hs[i], tolerance tol, and
 * fills info[i] (may be NULL; t_solve_ms is the whole batch's time).  Within
 * a problem the right-hand sides go through in groups of its build's nrhs.
 * nstreams <= 0 (and every handle built for PCG): one graph for the batch --
 * each problem's group of CG iterations is captured once, one batch graph
 * holds those of all iterating problems, and one launch advances every
 * problem; the host reads all residual histories with one synchronisation
 * per launch.  nstreams = 0: one batch graph, the groups one after another;
 * nstreams = -q (q <= 16): the problems dealt to q streams (largest first,
 * round-robin), one batch graph per stream, launched together.
 * nstreams > 0 (or another method): the problems are
 * spread over that many private streams (at most 16), one host thread each,
 * so the latency-bound coarse levels of different problems overlap.  Each handle's stream is ordered before and
 * after the batch; the call returns when all are done.  Handles must be
 * distinct (a handle is not thread-safe).  Returns the worst status.  Zero
 * Dirichlet data. */
hdg_status hdg_solve_batch(int nprob, const hdg_handle* hs, const double* const* rhs, int rhs_kind,
                           const int* nrhs, double tol, double* const* lambda, hdg_solve_info* info,
                           int nstreams);

/* Autotuner: times a few outer iterations of every candidate layout of the
 * work - coarsest macro grid (2, 8, 16) x right-hand-side group size (1, 2,
 * 4, ... <= nrhs) - on top of `base` (NULL: defaults), then, on the fastest
 * of those, the tile shapes of the kernels (one or four lanes per
 * macro-element in the transition kernels, two-phase instead of strip apply
 * on the finest level; variant bits); builds the handle with the fastest per
 * right-hand side and iteration, and returns it in *best (and that time in
 * microseconds in *us_per_rhs_it when not NULL). */
hdg_status hdg_autotune(hdg_handle h, const hdg_mg_opts* base, int nrhs, hdg_mg_opts* best, double* us_per_rhs_it);

/* hdg_rhs for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops): same arguments, result and errors as
 * hdg_rhs, but the per-element load staging lives in a fixed device array of
 * the library (64 MiB per GPU, held until the process ends) instead of
 * memory the handle allocated, and the call allocates nothing.  Supports
 * N_T ((k+1)^d + 2d (k+1)^(d-1)) <= 8 Mi doubles (e.g. 256 x 256 elements up
 * to k = 6, 512 x 512 up to k = 2); larger problems return
 * HDG_ERR_UNSUPPORTED.  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (several streams or threads) race. */
hdg_status hdg_rhs_noalloc(hdg_handle h, const double* rhs, int rhs_kind, const double* g_dirichlet, double* g);

/* Local recovery (q, u) = L_T^-1 (R_T Lambda_T + [0; b_T]) element by
 * element (Sec. 2); for the IPDG schemes u_T = L_T^-1 (R_T Lambda_T + b_T)
 * and q_T = -kappa_T grad u_T at the nodes.  Needs store_recovery at setup. */
hdg_status hdg_reconstruct(hdg_handle h, const double* lambda, const double* rhs, int rhs_kind,
                           const double* g_dirichlet, double* u, double* q);

/* Adjoint gradient: given the forward flux q_fwd [N_T][d][(k+1)^d] and the
 * misfit derivative dJdu in load form ([N_T][(k+1)^d], j_T = dJ/du_T),
 * solve the adjoint trace system (the forward operator with load j), recover
 * q*, and return grad[T] = dJ/d(log kappa_T) = -(q*_T)^T A_T q_T, A_T the
 * kappa^-1 weighted mass.  Derived from eqs. HDG and HDG_flux. */
/* (HDG handles with a scalar tau only; others get HDG_ERR_UNSUPPORTED.) */
hdg_status hdg_adjoint(hdg_handle h, const double* dJdu, const double* q_fwd, double tol,
                       double* grad_log_kappa, hdg_solve_info* info);

/* M_T u_T per element (the volume mass matrix), to turn nodal misfits into
 * loads: out[N_T][(k+1)^d]. */
hdg_status hdg_mass_apply(hdg_handle h, const double* u, double* out);

/* Inspection: y = A_l x on level l (0 = finest), precision per HDG_FP64/FP32. */
hdg_status hdg_level_apply(hdg_handle h, int level, const void* x, void* y, int precision);

/* Inspection: m steps of the build's smoother on A_l e = r from e = 0
 * (Chebyshev: m must be the level's sweep count, the polynomial's degree). */
hdg_status hdg_level_smooth(hdg_handle h, int level, const void* r, void* e, int sweeps, int precision);

/* Inspection: copy the element-form local matrices of level l
 * ([N_macro][n_loc][n_loc] row-major, local DOFs ordered by face slot
 * x-,x+,y-,y+,(z-,z+) then node) into out (device, double). */
hdg_status hdg_level_export(hdg_handle h, int level, double* out);

/* Inspection: time every launch of the finest-level trace kernels with HIP
 * events recorded on the handle's stream, from hdg_profile_begin until
 * hdg_profile_read.  kernel = 2 * mode + precision, mode 0 apply y = A x,
 * 1 residual b - A x, 2 block-Jacobi sweep x + D^-1 (b - A x), 3 residual
 * restricted to P1 (J_N^T), 6 the sweep inside CG's preconditioner that also
 * forms the r.z partials; precision HDG_FP64 / HDG_FP32; or kernel = 14 +
 * mode for the finest level of the mixed cycle with FP64 vectors over FP32
 * operator blocks (3D); or kernel = 21 + 2 * t + precision for the transfer
 * kernels of the fused 2D path, t = 0 hpre (interior residual, local
 * correction, restriction share) / 1 hsum (coarse residual and first coarse
 * Jacobi step) / 2 hpost (prolongation and post correction), all three on
 * the first h-transition level, t = 3 the p-prolongation on the finest
 * level.  Returns the number of launches, their summed duration, and the
 * algorithmic HBM bytes of one launch (stored face-major matrix blocks,
 * face-block inverses, macro-element blocks and each vector entry read or
 * written once). */
hdg_status hdg_profile_begin(hdg_handle h);
hdg_status hdg_profile_read(hdg_handle h, int kernel, long long* launches, double* total_ms,
                            double* bytes_per_launch);

enum {
  HDG_Q_NT = 0, HDG_Q_NLAMBDA = 1, HDG_Q_NLEVELS = 2, HDG_Q_NV = 3, HDG_Q_NQ = 4,
  HDG_Q_LEVEL_NLAMBDA = 100, /* + level */
  HDG_Q_LEVEL_N = 200,       /* + level: macro-elements per direction */
  HDG_Q_LEVEL_NE = 300,      /* + level: DOFs per face */
  HDG_Q_DEVICE_BYTES = 400,
  HDG_Q_GRID_TAIL = 401      /* first level of the persistent coarse cycle, FP64 cycle (-1: not used) */
};
hdg_status hdg_query(hdg_handle h, int what, long long* out);

/* GLL nodes (k+1 values on [0,1]) and Gauss points (k+2 values) used by the
 * library, written to host arrays. */
hdg_status hdg_reference_nodes(int k, double* gll, double* gauss);

hdg_status hdg_destroy(hdg_handle h);
const char* hdg_status_string(hdg_status s);

#ifdef __cplusplus
}
#endif
#endif /* HDG_H */

/*
 * p2m.h -- C ABI of libp2m.so: particle<->mesh assignment on periodic P1 meshes
 * for AMD Instinct MI355X (gfx950).
 *
 * Method: D. Duque and P. Espanol, "Assignment of fields from particles to mesh",
 * arXiv 1610.05258.  Particle->mesh ("P2M") finds nodal values Abar_i from particle
 * values A_mu; mesh->particle ("M2P") finds particle values from nodal ones
 * (Sec. 2).  The methods are the rows of Table 1: delta (Sec. 2.2), FLIP and PIC
 * (Sec. 2.3) and the "mass" assignment (Sec. 2.4).
 *
 * Integrals.  Every integral of the method is evaluated with the particle
 * quadrature int f = sum_mu v_mu f(r_mu) that the paper uses for int A (Sec. 2.1)
 * and for the FLIP volume (Sec. 2.3, eq. (12)).  The mass matrix of Sec. 2.4 is
 * therefore M_ij = sum_mu v_mu psi_i(r_mu) psi_j(r_mu) and the mass assignment
 * solves M Abar = b with b_i = sum_mu v_mu A_mu psi_i(r_mu).
 *
 * Mesh.  A problem is one periodic structured mesh: nx (1D) or nx*ny (2D) nodes
 * on [0,lx) x [0,ly), node i (1D) at i*hx, node k = i + nx*j (2D) at (i*hx, j*hy),
 * hx = lx/nx, hy = ly/ny.  Cells are indexed like their lower-left node.  In 2D
 * every cell is split by its "/" diagonal (lower-left to upper-right) into two
 * triangles; psi_i is the P1 hat of node i.
 *
 * Conventions shared by every entry point.
 *  - All array arguments are DEVICE pointers, allocated and owned by the caller;
 *    the library never frees them and never allocates device memory inside a
 *    call.  Scratch memory is the caller's workspace (p2m_workspace_size).
 *  - Layouts are structure-of-arrays; a field index is always the outer index:
 *    values[f*np + mu], nodal[f*nnodes + k].
 *  - Every call is asynchronous on `stream` (a hipStream_t passed as void*,
 *    NULL = the null stream) and returns synchronously only argument and launch
 *    errors.  Problems found in the data on the device are written as flags into
 *    a p2m_report that lives in device memory.
 *  - Indices are int32: np < 2^31 and nnodes < 2^31, else P2M_ERR_UNSUPPORTED.
 *  - dtype selects FP32 or FP64 for positions, volumes, values and nodal arrays
 *    of a call; all of them share it.
 *  - A context must not be used from two host threads at once.
 */
#ifndef P2M_H
#define P2M_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    P2M_OK = 0,
    P2M_ERR_INVALID_ARG = 1,   /* NULL pointer, dim not 1/2, n < 2, F not in [1,8], bad enum */
    P2M_ERR_UNSUPPORTED = 2,   /* sizes beyond int32 indexing or beyond a kernel's limits */
    P2M_ERR_WORKSPACE = 3,     /* ws NULL or ws_bytes smaller than p2m_workspace_size */
    P2M_ERR_RANGE = 4,         /* lx, ly not > 0, or tol not > 0 */
    P2M_ERR_NONFINITE = 5,     /* lx, ly or tol not finite */
    P2M_ERR_HIP = 6,           /* a HIP runtime call or kernel launch failed */
    P2M_ERR_SCRATCH = 7        /* p2m_mass_assign_noalloc: the problem needs more workspace
                                  than the static scratch holds (P2M_SCRATCH_BYTES) */
} p2m_status;

/* Report flags (p2m_report.flags).  Output contents are defined for every flag:
 * ORPHAN nodes get 0; NOT_CONVERGED returns the last iterate; RANGE / NONFINITE
 * particles are left out of P2M and get NaN in M2P. */
enum {
    P2M_FLAG_ORPHAN = 1u << 0,           /* some node has w_i == 0 (Sec. 2.3: vanishing FLIP volume) */
    P2M_FLAG_NOT_CONVERGED = 1u << 1,    /* mass solve stopped above tol (maxit / max_refine) */
    P2M_FLAG_BREAKDOWN = 1u << 2,        /* CG met p.Mp <= 0 or a non-finite scalar */
    P2M_FLAG_RANGE = 1u << 3,            /* some position outside [0, L + h) */
    P2M_FLAG_NONFINITE = 1u << 4,        /* some position is NaN or infinite */
    P2M_FLAG_LEARNED_FALLBACK = 1u << 5, /* learned start was worse than FLIP and was replaced */
    P2M_FLAG_BIN_TIMEOUT = 1u << 6,      /* the binning scan's bounded wait for another workgroup
                                            ended: the binning is discarded (every cell empty:
                                            cell_start all 0, perm all -1), so P2M results are 0
                                            (orphans) and M2P is unaffected; retry the call */
    P2M_FLAG_TRIANGULATION = 1u << 7     /* p2m_x2d_*: the particle triangulation is incomplete
                                            (a Voronoi cell not closed within the search radius,
                                            more than P2M_X2D_MAXDEG neighbours, two particles at
                                            one position, or neighbour lists that disagree); the
                                            values that depend on it are NaN */
};

typedef enum { P2M_F32 = 0, P2M_F64 = 1 } p2m_dtype;

/* One periodic P1 problem (64 bytes). */
typedef struct {
    int32_t dim;          /* 1 or 2 */
    int32_t nx, ny;       /* nodes (= cells) per axis, >= 2; ny is ignored (treated as 1) in 1D */
    int32_t dtype;        /* p2m_dtype of x, y, vol and of the values / nodal arrays of the call */
    double lx, ly;        /* box [0,lx) x [0,ly); ly ignored in 1D */
    int64_t np;           /* number of particles (may be 0) */
    const void* x;        /* [np] positions; valid positions satisfy 0 <= x*(nx/lx) < nx+1 */
    const void* y;        /* [np] (2D only, NULL in 1D) */
    const void* vol;      /* [np] particle volumes v_mu (> 0), or NULL for uniform lx*ly/np */
} p2m_problem;

typedef enum {
    P2M_DELTA = 0,        /* 1D only: Abar_i = particle interpolant at node i, eq. (9) */
    P2M_FLIP = 1,         /* Abar_i = b_i / w_i, eqs. (11)-(12) */
    P2M_PIC = 2           /* Abar_i = b_i / v_i with v_i = hx (1D) or hx*hy (2D), eqs. (11), (5) */
} p2m_assign_kind;

typedef enum {
    P2M_START_FLIP = 0,     /* x0 = b/w (the FLIP values; equal to delta for regular particles, Sec. 3.1) */
    P2M_START_ZERO = 1,
    P2M_START_USER = 2,     /* x0 read from nodal_inout */
    P2M_START_LEARNED = 3,  /* the learned warm start (p2m_set_learned); 2D FP32 only */
    P2M_START_DELTA1D = 4   /* 1D only: the delta assignment as x0 */
} p2m_start;

/* Mass-solve options (32 bytes).  The solve is conjugate gradients on M Abar = b,
 * restarted from the true residual r = b - M x evaluated in FP64 ("outer"
 * iterations, iterative refinement).  It stops when ||r||_2 / ||b||_2 <= tol for
 * every field (b == 0 gives x == 0). */
typedef struct {
    double tol;           /* relative FP64 residual target, > 0 (e.g. 1e-6) */
    double inner_rtol;    /* each inner CG solve reduces its residual by this factor (0: to tol) */
    int32_t maxit;        /* cap on CG iterations per field, summed over outer iterations */
    int32_t max_refine;   /* cap on FP64 residual evaluations after the first (>= 0) */
    int32_t start;        /* p2m_start */
    int32_t reserved;     /* must be 0 */
} p2m_solve_opts;

/* Per-call report, written on the device (144 bytes, device memory, caller-owned). */
typedef struct {
    int32_t iters[8];          /* CG iterations per field */
    int32_t refines[8];        /* FP64 residual evaluations per field */
    double rel_residual[8];    /* final FP64 ||b - M x||_2 / ||b||_2 per field */
    uint32_t flags;            /* P2M_FLAG_* */
    int32_t n_orphan;          /* nodes with w_i == 0 */
    int32_t n_invalid;         /* particles left out (range / non-finite) */
    int32_t reserved;
} p2m_report;

/* Human-readable name of a status code (static storage). */
const char* p2m_status_string(p2m_status s);

/* Create a context on HIP device `device` (queries the device; allocates nothing
 * on it).  Destroy releases the context. */
p2m_status p2m_create(void** ctx, int device);
p2m_status p2m_destroy(void* ctx);

/* Mass-solve kernels.  Every one solves the same system to the same tolerance;
 * their rounding differs, except that the resident and the tile-streaming kernels
 * give identical bits (the same per-tile arithmetic and reduction order).
 *   P2M_SOLVER_AUTO       the register-resident kernel where it applies (2D FP32,
 *                         F <= 3, at most one 128 x 32 node tile per workgroup that
 *                         fits the device at once), else the tile-streaming
 *                         kernel (2D FP32, F <= 3, any size), else the streaming
 *                         kernel; a tuned plan of the problem's shape class
 *                         (p2m_tune) overrides this choice
 *   P2M_SOLVER_STREAMING  grid-synchronised streaming kernel (any problem)
 *   P2M_SOLVER_RESIDENT   register-resident kernel where it applies (as AUTO)
 *   P2M_SOLVER_TILES      tile-streaming kernel where it applies
 *   P2M_SOLVER_RESIDENT_CHEB
 *                         the register-resident kernel with a degree-2 Chebyshev
 *                         polynomial preconditioner, u = (c0 + c1 D^-1 M) D^-1 r,
 *                         instead of the diagonal one (D = diag M): the same system
 *                         and tolerance in fewer iterations, one grid barrier each;
 *                         where it does not apply, as AUTO.  The tuner tries it;
 *                         AUTO itself keeps the diagonal preconditioner. */
enum { P2M_SOLVER_AUTO = 0, P2M_SOLVER_STREAMING = 1, P2M_SOLVER_RESIDENT = 2, P2M_SOLVER_TILES = 3,
       P2M_SOLVER_RESIDENT_CHEB = 4 };

/* Context options (p2m_set_option).
 *   P2M_OPT_SOLVER     a P2M_SOLVER_* value (default AUTO); anything but AUTO forces
 *                      that kernel where it applies, tuned plans notwithstanding
 *   P2M_OPT_PLANS      1 (default): apply tuned plans; 0: ignore them
 *   P2M_OPT_SCAN_SPIN  bound on the polls of the binning scan's wait for a
 *                      preceding workgroup's prefix (0: the default, 2^26); a
 *                      negative value ends every such wait at once, which
 *                      raises P2M_FLAG_BIN_TIMEOUT on any mesh of more than 2048
 *                      cells (for testing the timeout handling)
 *   P2M_OPT_SOLVE_SPIN bound on the polls of a mass solve's grid-barrier wait
 *                      (0: the default, 2^22); a negative value ends every such
 *                      wait at once: a solve whose grid has more than one
 *                      workgroup then stops at its first barrier with
 *                      P2M_FLAG_BREAKDOWN | P2M_FLAG_NOT_CONVERGED and the last
 *                      FP64 solution it held as the result (for testing the
 *                      timeout handling; every kernel still runs to its end)
 *   P2M_OPT_FFT        1 (default): the circulant mesh systems of p2m_ns_step and
 *                      the paper-exact 2D mass P2M are solved directly by the 2D
 *                      discrete Fourier transform when both mesh sides are at most
 *                      1024 or powers of two up to 2048; 0: always by the iterative
 *                      mass-matrix solver */
enum { P2M_OPT_SOLVER = 0, P2M_OPT_PLANS = 1, P2M_OPT_SCAN_SPIN = 2, P2M_OPT_SOLVE_SPIN = 3,
       P2M_OPT_FFT = 4 };
p2m_status p2m_set_option(void* ctx, int32_t option, int32_t value);

/* Bytes of workspace that every call below needs for this problem and field count
 * (the maximum over the entry points, so one workspace serves all of them).
 * The workspace must be 256-byte aligned device memory. */
p2m_status p2m_workspace_size(void* ctx, const p2m_problem* prob, int32_t nfields, size_t* bytes);

/* Stable binning of the particles by cell (the locality step of every P2M).
 * perm[k] = original index of the k-th valid particle in (cell, original index)
 * order, perm[k] = -1 for k >= number of valid particles; cell_start[c] = index in
 * perm of the first particle of cell c, cell_start[ncells] = number of valid
 * particles (ncells = nx or nx*ny).  Bit-exact and deterministic. */
p2m_status p2m_bin(void* ctx, const p2m_problem* prob, int32_t* perm, int32_t* cell_start,
                   p2m_report* rep, void* ws, size_t ws_bytes, void* stream);

/* Scatter of the particle-quadrature system (Sec. 2.3 eqs. (11)-(12), Sec. 2.4):
 *   b[f*nn + i] = sum_mu v_mu A_f,mu psi_i(r_mu)
 *   w[i]        = sum_mu v_mu psi_i(r_mu)
 *   coef (optional, may be NULL): the symmetric stencil of M,
 *     2D: coef[0*nn+k] = M(k,k), coef[1*nn+k] = M(k,k+x), coef[2*nn+k] = M(k,k+y),
 *         coef[3*nn+k] = M(k,k+x+y)  (neighbour indices periodic);
 *     1D: coef[0*nn+k] = M(k,k), coef[1*nn+k] = M(k,k+1).
 * Each sum runs over the particles of a cell in binned order and then over the
 * cells around a node in a fixed order: deterministic, no global float atomics. */
p2m_status p2m_assemble(void* ctx, const p2m_problem* prob, const void* values, int32_t nfields,
                        void* b, void* w, void* coef, p2m_report* rep,
                        void* ws, size_t ws_bytes, void* stream);

/* Particle->mesh by delta (1D), FLIP or PIC (Table 1).  nodal_out is [F][nnodes];
 * orphan nodes (w_i == 0) get 0 under FLIP and raise P2M_FLAG_ORPHAN. */
p2m_status p2m_assign(void* ctx, const p2m_problem* prob, p2m_assign_kind kind, const void* values,
                      int32_t nfields, void* nodal_out, p2m_report* rep,
                      void* ws, size_t ws_bytes, void* stream);

/* Mesh->particle interpolation (Sec. 2.2 eq. (10), the M2P of delta, FLIP and
 * mass-delta in Table 1): values_out[f*np + mu] = sum_i nodal[f*nn + i] psi_i(r_mu),
 * in the caller's particle order.  Needs no workspace (ws may be NULL); with a
 * workspace of at least nfields * nnodes elements (256-byte aligned device
 * memory, contents overwritten), 2D problems with 2 to 4 fields first copy the
 * nodal values node-major into it and read each triangle corner's fields with
 * one load.  The values are the same either way. */
p2m_status p2m_interpolate(void* ctx, const p2m_problem* prob, const void* nodal, int32_t nfields,
                           void* values_out, p2m_report* rep, void* ws, size_t ws_bytes, void* stream);

/* Mass assignment (Sec. 2.4 eqs. (13), (19); Table 1 mass rows): assemble M and b
 * and solve M Abar_f = b_f for every field with the precision split described at
 * p2m_solve_opts (FP32 arithmetic when dtype is F32, FP64 residuals and dot
 * products).  Orphan nodes (w_i == 0) are solved as Abar_i = 0.  nodal_inout is
 * [F][nnodes]: read as the start when opts->start == P2M_START_USER, always
 * written with the result.  With P2M_START_LEARNED (2D FP32, parameters set with
 * p2m_set_learned) the network proposes the start; a field whose proposed start
 * has a larger FP64 residual ||b - M x0|| than the FLIP start is started from
 * FLIP instead and P2M_FLAG_LEARNED_FALLBACK is raised.  rep is required. */
p2m_status p2m_mass_assign(void* ctx, const p2m_problem* prob, const void* values, int32_t nfields,
                           const p2m_solve_opts* opts, void* nodal_inout, p2m_report* rep,
                           void* ws, size_t ws_bytes, void* stream);

/* Mass assignment that allocates nothing, for callers that cannot allocate
 * device memory or pass a workspace (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  The same computation and
 * the same kernels as p2m_mass_assign, bit for bit, with the workspace taken
 * from a static device array of P2M_SCRATCH_BYTES (64 MiB) that the library
 * holds on every device it runs on until the process ends; its device address
 * is looked up once per device when a context is created.  The caller still
 * passes values, nodal_inout and rep (device memory, as for p2m_mass_assign).
 * Returns P2M_ERR_SCRATCH, launching nothing, when p2m_workspace_size of the
 * problem exceeds P2M_SCRATCH_BYTES (for example 2D meshes of about 256 x 256
 * nodes at 8 particles per cell and F = 3 fit; 1024 x 1024 does not), and
 * P2M_ERR_HIP if the scratch's address could not be looked up.  Every call on
 * one device shares that device's scratch and leaves its contents behind (each
 * call clears what it needs cleared itself): calls that overlap on one device,
 * on different streams or from different host threads, race and must not be
 * issued. */
enum { P2M_SCRATCH_BYTES = 64 << 20 };
p2m_status p2m_mass_assign_noalloc(void* ctx, const p2m_problem* prob, const void* values,
                                   int32_t nfields, const p2m_solve_opts* opts, void* nodal_inout,
                                   p2m_report* rep, void* stream);

/* The solve step of p2m_mass_assign alone, for a system assembled by
 * p2m_assemble with the same problem and field count (b [F][nn], w [nn], coef
 * [4 or 2][nn] as documented there).  b and coef are modified in place: orphan
 * rows (w_i == 0) become identity rows with b_i = 0.  opts->start may be FLIP
 * (b/w), ZERO or USER (read from nodal_inout); DELTA1D needs the particles and is
 * P2M_ERR_UNSUPPORTED here.  Launches one solver kernel (after a report clear and,
 * for the tile solvers, a counter clear).  rep is required. */
p2m_status p2m_mass_solve(void* ctx, const p2m_problem* prob, int32_t nfields, void* b,
                          const void* w, void* coef, const p2m_solve_opts* opts, void* nodal_inout,
                          p2m_report* rep, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Paper-exact 1D assignment (Table 1 with the particle hats of Sec. 2: in 1D the
 * particle "triangulation" is the order of the particles along the periodic
 * segment; Sec. 3.1).  FP64 1D problems only (dtype P2M_F64, dim 1; prob->vol is
 * ignored: the particle volumes are those of eq. (4), v_mu = (x_{mu+1} -
 * x_{mu-1}) / 2 on the sorted particles).  Particles are ordered by wrapped
 * position, ties by particle number.  The integrals int A psi_j (P2M, mesh hats
 * psi_j, A the particle interpolant of eq. (1)) and int Abar psi_mu (M2P,
 * particle hats, Abar the mesh interpolant of eq. (3)) are evaluated either
 * exactly (P2M_QUAD_EXACT: breakpoints of both interpolants merged, Simpson's
 * rule exact on every piece) or with the Appendix-B rule (P2M_QUAD_APPB: on
 * every gap of the target hats, the parabola through the source interpolant at
 * both ends and the midpoint, integrated exactly).  Mass systems use the
 * consistent mass matrices (mesh: 2h/3 and h/6; particles: (g_{mu-1} + g_mu)/3
 * and g_mu/6 with g_mu = x_{mu+1} - x_mu) and are solved by the FP64 streaming
 * CG to opts->tol.  Each call synchronises `stream` once, after binning (to
 * size the particle-order arrays).  Particles that cannot be located are left
 * out (P2M) and get NaN (M2P); at least one located particle is needed for the
 * mass and lumped kinds and for delta.
 * --------------------------------------------------------------------------- */
typedef enum { P2M_QUAD_EXACT = 0, P2M_QUAD_APPB = 1 } p2m_quad;
typedef enum {
    P2M_X1D_DELTA = 0,   /* P2M: Abar_i = A(x_i), eq. (9);  M2P: Abar(x_mu), eq. (10) */
    P2M_X1D_FLIP = 1,    /* P2M only: eqs. (11)-(12) with the volumes of eq. (4) */
    P2M_X1D_PIC = 2,     /* P2M only: eq. (11) with v_i = h, eq. (5) */
    P2M_X1D_MASS = 3,    /* P2M: m^-1 int A psi_j (mass-delta and full mass, Table 1);
                            M2P: m_part^-1 int Abar psi_mu, eq. (20) (full mass) */
    P2M_X1D_LUMPED = 4   /* P2M: (1/h) int A psi_i;  M2P: (1/v_mu) int Abar psi_mu, eq. (17) */
} p2m_x1d_kind;

/* Workspace bytes of the three calls below for this problem and field count. */
p2m_status p2m_x1d_workspace_size(void* ctx, const p2m_problem* prob, int32_t nfields,
                                  size_t* bytes);
/* Particle -> mesh: nodal_out [F][nx] (device).  opts is used by P2M_X1D_MASS (NULL:
 * tol 1e-14); rep (device, required) receives the solve's report. */
p2m_status p2m_x1d_assign(void* ctx, const p2m_problem* prob, int32_t kind, int32_t quad,
                          const void* values, int32_t nfields, const p2m_solve_opts* opts,
                          void* nodal_out, p2m_report* rep, void* ws, size_t ws_bytes,
                          void* stream);
/* Mesh -> particle (kind DELTA, MASS or LUMPED): values_out [F][np] in caller order. */
p2m_status p2m_x1d_interpolate(void* ctx, const p2m_problem* prob, int32_t kind, int32_t quad,
                               const void* nodal, int32_t nfields, const p2m_solve_opts* opts,
                               void* values_out, p2m_report* rep, void* ws, size_t ws_bytes,
                               void* stream);
/* The particle volumes of eq. (4), vol_out [np] in caller order (NaN: not located). */
p2m_status p2m_x1d_volumes(void* ctx, const p2m_problem* prob, void* vol_out, p2m_report* rep,
                           void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Paper-exact 2D assignment (Table 1 with the particle hats of Sec. 3.2: P1 hats
 * on the periodic Delaunay triangulation of the particles; the Appendix-B rule
 * for every overlap integral).  FP64 2D problems only (dtype P2M_F64, dim 2;
 * prob->vol is ignored: the particle volumes are v_mu = int psi_mu, a third of the
 * area of the triangles around mu).  Positions must be distinct.
 *
 * The triangulation is built on the device: every particle clips its Voronoi cell
 * against the particles of the surrounding cells of the mesh, ring by ring, until
 * no particle outside the searched rings can cut it (twice the farthest Voronoi
 * vertex is within the searched radius; at most 8 rings); its Delaunay neighbours
 * are the particles whose bisectors bound the cell, counter-clockwise.  Each
 * triangle must then appear in the lists of its three vertices.
 *   delta P2M      Abar_i = A(r_i): the particle interpolant of eq. (1) at the node,
 *                  found by a walk through the triangulation from the nearest
 *                  particle (eq. (9)).
 *   FLIP / PIC     eqs. (11)-(12) / eq. (11) with the volumes above.
 *   mass P2M       m Abar = b, b_j = int A psi_j by the Appendix-B rule on the mesh
 *                  triangles (A at the vertices and edge midpoints, the quadratic
 *                  through them integrated exactly against psi_j); m the
 *                  consistent mesh mass matrix (hx hy / 2 on the diagonal, hx hy /
 *                  12 to the six neighbours of the "/" split); mass-delta and full
 *                  mass P2M of Table 1.
 *   lumped P2M     b_i / (hx hy) (eq. (17)).
 *   delta M2P      the mesh interpolant at the particle (eq. (10)).
 *   mass M2P       m_part Abarbar = c, c_nu = int Abar psi_nu by the Appendix-B
 *                  rule on the particle triangles, m_part the consistent particle
 *                  mass matrix (|T|/6 on the diagonal, |T|/12 off it, summed over
 *                  the triangles), eq. (20) (full mass).
 *   lumped M2P     c_nu / v_nu (eq. (17)).
 * The mesh mass system is solved directly by a 2D FFT in FP64 when both sides are
 * at most 1024 or powers of two up to 2048 (it is circulant; the report then shows
 * 0 iterations),
 * otherwise, like the particle mass system, by the FP64 streaming CG to opts->tol
 * (NULL: 1e-14).  Kinds are those of p2m_x1d_kind; the quadrature is always the
 * Appendix-B rule.
 * Each call synchronises `stream` once, after binning.  Particles that cannot be
 * located are left out (P2M) and get NaN (M2P). rep (device) is required.
 * --------------------------------------------------------------------------- */
#define P2M_X2D_MAXDEG 32

/* Workspace bytes of the calls below for this problem and field count. */
p2m_status p2m_x2d_workspace_size(void* ctx, const p2m_problem* prob, int32_t nfields,
                                  size_t* bytes);
/* The triangulation, in caller particle numbers: deg_out [np] (0: not located or
 * failed), nbr_out [np][P2M_X2D_MAXDEG] the neighbours counter-clockwise (-1 past
 * deg), shift_out [np][P2M_X2D_MAXDEG] the image of each neighbour, packed as
 * (sx + 128) | (sy + 128) << 8: neighbour j of mu sits at
 * (x_nbr + sx lx, y_nbr + sy ly).  Consecutive neighbours j, j+1 (cyclic) span
 * the counter-clockwise triangle (mu, nbr_j, nbr_j+1). */
p2m_status p2m_x2d_triangulation(void* ctx, const p2m_problem* prob, int32_t* deg_out,
                                 int32_t* nbr_out, int32_t* shift_out, p2m_report* rep, void* ws,
                                 size_t ws_bytes, void* stream);
/* The particle volumes int psi_mu, vol_out [np] in caller order (NaN: not located). */
p2m_status p2m_x2d_volumes(void* ctx, const p2m_problem* prob, void* vol_out, p2m_report* rep,
                           void* ws, size_t ws_bytes, void* stream);
/* Particle -> mesh (kind DELTA, FLIP, PIC, MASS or LUMPED): nodal_out [F][nx ny]. */
p2m_status p2m_x2d_assign(void* ctx, const p2m_problem* prob, int32_t kind, const void* values,
                          int32_t nfields, const p2m_solve_opts* opts, void* nodal_out,
                          p2m_report* rep, void* ws, size_t ws_bytes, void* stream);
/* Mesh -> particle (kind DELTA, MASS or LUMPED): values_out [F][np] in caller order. */
p2m_status p2m_x2d_interpolate(void* ctx, const p2m_problem* prob, int32_t kind,
                               const void* nodal, int32_t nfields, const p2m_solve_opts* opts,
                               void* values_out, p2m_report* rep, void* ws, size_t ws_bytes,
                               void* stream);
/* One Table 1 pair at one set of positions (the per-step projection of Sec. 3.2):
 * p2m_x2d_assign of kind_p2m into nodal_out [F][nx ny], then p2m_x2d_interpolate
 * of kind_m2p (DELTA, MASS or LUMPED) of nodal_out into values_out [F][np], with
 * one binning and one triangulation.  reps (device) holds two reports: reps[0]
 * the binning and triangulation flags and the P2M solve, reps[1] the M2P solve.
 * The results equal those of the two separate calls. */
p2m_status p2m_x2d_round_trip(void* ctx, const p2m_problem* prob, int32_t kind_p2m,
                              int32_t kind_m2p, const void* values, int32_t nfields,
                              const p2m_solve_opts* opts, void* nodal_out, void* values_out,
                              p2m_report* reps, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Particle fluid solver: the Taylor-Green vortex sheet computation of Sec. 3.3
 * (incompressible Navier-Stokes, particles carrying the velocity, space derivatives
 * on the mesh).  The paper names only a standard splitting approach with mid-point
 * time integration; the step below is that reading, for equal-order P1 velocity
 * and pressure on the problem's periodic mesh (2D, FP32, square cells lx/nx ==
 * ly/ny):
 *   1. P2M of the particle velocities vel [2][np] (u then v) with FLIP
 *      (P2M_NS_FLIP, Sec. 2.3) or the mass assignment (P2M_NS_MASS, Sec. 2.4):
 *      nodal Ubar;
 *   2. implicit viscous step (M_L + dt nu K) U* = M_L Ubar, K the P1 stiffness
 *      matrix (the five-point Laplacian on this mesh), M_L = h^2 the lumped P1 mesh
 *      mass;
 *   3. pressure K p = -(1/dt) D U*, (D U)_i = int psi_i div U_h, with node 0 held at
 *      p = 0 (the system is singular in the constants);
 *   4. projection U^{n+1} = U* - dt M_L^-1 G p, (G p)_i = int psi_i grad p_h;
 *   5. M2P: vel <- U^{n+1} interpolated at the particles (Sec. 2.2 eq. (10));
 *   6. mid-point advection r* = r + (dt/2) vel, r <- r + dt U^{n+1}(r*), each
 *      coordinate wrapped into [0, L) in FP64 and rounded once.
 * Step 1's mass system is solved by the mass-matrix solver (FP32 CG, FP64
 * residuals and refinement) to opts->tol from opts->start, which must be
 * P2M_START_FLIP or P2M_START_ZERO.  The systems of steps 2 and 3 are circulant:
 * when nx and ny are powers of two (at most 2048) they are solved exactly by 2D FFT
 * in FP64 (zero-mean pressure instead of the held node; reports 1 and 2 then show
 * no iteration), otherwise by the same solver from b / diag, the pressure solve with
 * an iteration cap of at least 64 per mesh side.
 * --------------------------------------------------------------------------- */
typedef enum { P2M_NS_FLIP = 0, P2M_NS_MASS = 1 } p2m_ns_assign;

/* Workspace bytes of p2m_ns_step for this problem (the F = 2 assignment workspace
 * plus 20 floats per node, and 64 bytes per node of transform buffers when both
 * sides are powers of two). */
p2m_status p2m_ns_workspace_size(void* ctx, const p2m_problem* prob, size_t* bytes);
/* One time step dt with kinematic viscosity nu (dt > 0, nu >= 0, finite).
 *   vel       [2][np] FP32, in: the particle velocities at prob->x, prob->y;
 *             out: the new ones (step 5)
 *   x_out, y_out [np] FP32: the advected positions; may be prob->x, prob->y
 *   mesh_vel  [2][nn] FP32 out: U^{n+1}, or NULL (then kept in the workspace)
 *   reps      [3] device reports: 0 = binning, step 1 (its solve for P2M_NS_MASS),
 *             M2P and advection (invalid particles: flags, NaN outputs); 1 = the
 *             viscous solve; 2 = the pressure solve (iterations, refinements,
 *             relative residual per component, NOT_CONVERGED / BREAKDOWN)
 * Errors: P2M_ERR_INVALID_ARG (NULL ctx / reps / arrays, bad assign),
 * P2M_ERR_NONFINITE / P2M_ERR_RANGE (dt, nu, opts), P2M_ERR_UNSUPPORTED (not 2D
 * FP32 with square cells, another start), P2M_ERR_WORKSPACE, P2M_ERR_HIP. */
p2m_status p2m_ns_step(void* ctx, const p2m_problem* prob, int32_t assign, double dt, double nu,
                       const p2m_solve_opts* opts, void* vel, void* x_out, void* y_out,
                       void* mesh_vel, p2m_report* reps, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Batches: many independent problems in one launch.
 *
 * A batch is nprob independent 2D FP32 problems (each its own mesh size, box,
 * particles and volumes) with the same field count F, 1 <= F <= 3, nprob <= 128
 * and nprob * F <= 256.  Every instance is mass-assigned exactly as
 * p2m_mass_assign would do it alone with the register-resident solver
 * (P2M_OPT_SOLVER 0 or 2): the same binning, the same scatter sums and the same
 * solver arithmetic in the same order, so each instance's nodal values and
 * report equal the single-problem ones bit for bit, whatever the other
 * instances are.
 *
 * The whole batch is one HIP graph: clears, binning, scatter of all instances
 * and one persistent solve kernel over the solver tiles of all instances (tiles
 * are shared out over at most one workgroup per compute unit; the kernel's
 * grid-wide barriers rely on all its workgroups being resident, which holds on a
 * device not shared with other work, and its waits are bounded: a timed-out wait
 * ends the solve with P2M_FLAG_BREAKDOWN | P2M_FLAG_NOT_CONVERGED).
 *
 * The context caches the graph of the last batch.  A call whose instance table
 * (problems, particle / value / nodal pointers), F, options, workspace and
 * reports are those of the previous call relaunches the cached graph (one
 * hipGraphLaunch, nothing else); any other call builds a new graph first, which
 * copies the instance table and tile maps (host memory) to the head of the
 * workspace and synchronises `stream` once.
 * --------------------------------------------------------------------------- */

/* Workspace bytes of p2m_mass_assign_batched for this batch (256-byte aligned
 * device memory).  P2M_ERR_UNSUPPORTED for problems that are not 2D FP32, for
 * F > 3, nprob > 128, nprob * F > 256, or batches beyond int32 indexing or the
 * solve kernel's tile capacity (32 solver tiles of 128 x 32 nodes per compute
 * unit). */
p2m_status p2m_batch_workspace_size(void* ctx, const p2m_problem* probs, int32_t nprob,
                                    int32_t nfields, size_t* bytes);

/* Mass assignment of every instance of a batch (Sec. 2.4, as p2m_mass_assign).
 *   probs        host array [nprob] of problems (dim 2, dtype P2M_F32)
 *   values       host array [nprob] of device pointers, values[k] is [F][np_k]
 *                (may be NULL when np_k == 0)
 *   opts         one set of options for all instances; start FLIP, ZERO or USER
 *   nodal_inout  host array [nprob] of device pointers, [F][nn_k] each: the start
 *                when opts->start == P2M_START_USER, always the result
 *   reps         device array [nprob] of reports, reps[k] for instance k (required)
 * Asynchronous on `stream` apart from the graph build described above. */
p2m_status p2m_mass_assign_batched(void* ctx, const p2m_problem* probs, int32_t nprob,
                                   const void* const* values, int32_t nfields,
                                   const p2m_solve_opts* opts, void* const* nodal_inout,
                                   p2m_report* reps, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Learned warm start (not part of the paper's method: a start vector for the
 * mass solve; the solve, its tolerance and the residual test are unchanged).
 *
 * Node features.  The receptive field of node i is the support of psi_i, the
 * four cells sharing the node: a = (ix, iy), b = (ix-1, iy), c = (ix-1, iy-1),
 * d = (ix, iy-1) (periodic).  Their particles are taken cell by cell in that
 * order, each cell in binned order (ascending original index), and the first
 * P2M_LEARNED_KMAX are kept; n counts them all.  A kept particle contributes
 * three inputs: its offset from the node in cell units, (xi - [cell b or c],
 * eta - [cell c or d]) from the FP64 locate, and (A - base) / s, where base =
 * b_i / w_i is the FLIP value (0 at an orphan) and s the RMS of A - base over the
 * kept particles.  Input 144 is min(n, 48) / 48; inputs of absent particles and
 * inputs 145..159 are 0.  A node is usable when 1 <= n <= 48, w_i > 0 and
 * s > 2^-20 max |A| over its kept particles.
 *
 * Network.  z1 = W1 x + b1, h1 = relu(z1), z2 = W2 h1 + b2, h2 = relu(z2),
 * z3 = W3 h2 + b3, h3 = relu(z3), y = W4 . h3 + b4.  W1..W3, x, h1, h2 are
 * rounded to BF16 (to nearest even) and multiplied on the matrix cores with
 * FP32 accumulation; biases, W4 and h3 are FP32.  The start value of a usable
 * node is base + s * y, of any other node base.
 *
 * Parameters: one FP32 device vector of P2M_LEARNED_NPARAM entries, in order
 * W1 [64][160] (row-major, columns 145..159 unused), b1 [64], W2 [64][64],
 * b2 [64], W3 [64][64], b3 [64], W4 [64], b4 [1].
 * --------------------------------------------------------------------------- */
enum {
    P2M_LEARNED_KMAX = 48,
    P2M_LEARNED_NIN = 160,
    P2M_LEARNED_HIDDEN = 64,
    P2M_LEARNED_NPARAM = 18689
};

/* Parameters used by P2M_START_LEARNED on this context (device pointer, read at
 * every call; NULL disables the learned start).  For callers that train a
 * network or load trained weights. */
p2m_status p2m_set_learned(void* ctx, const float* params);

/* Feature rows of nodes[0..nrows) (nodes NULL: every node, nrows = nnodes) of a
 * 2D FP32 problem: bins and scatters the particles (b and w), then writes
 *   x_out     [nrows][F][160] BF16 (2-byte elements, layout above),
 *   base_out  [nrows][F] the FLIP values, scale_out [nrows][F] s, or 0 where the
 *             node is not usable.
 * Needs the workspace of p2m_workspace_size. */
p2m_status p2m_learned_features(void* ctx, const p2m_problem* prob, const void* values,
                                int32_t nfields, const int32_t* nodes, int32_t nrows, void* x_out,
                                float* base_out, float* scale_out, p2m_report* rep, void* ws,
                                size_t ws_bytes, void* stream);

/* Network outputs y_out[r] of feature rows x [nrows][160] (BF16) with params. */
p2m_status p2m_learned_forward(void* ctx, const float* params, const void* x, int32_t nrows,
                               float* y_out, void* stream);

/* Workspace bytes of p2m_learned_train_step for a batch size. */
p2m_status p2m_learned_workspace_size(void* ctx, int32_t batch, size_t* bytes);

/* One training step on the rows rows[0..batch) of x [.][160] (BF16) with targets
 * target[row] (FP32): the loss (1/batch) sum (y - target)^2 goes to loss_out[0]
 * (device), its gradient to grad_out (device, P2M_LEARNED_NPARAM, may be NULL);
 * with apply != 0 one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected
 * with step >= 1, learning rate lr) updates params, adam_m and adam_v in place.
 * Deterministic: every sum has a fixed order. */
p2m_status p2m_learned_train_step(void* ctx, float* params, float* adam_m, float* adam_v,
                                  int32_t step, float lr, const void* x, const float* target,
                                  const int32_t* rows, int32_t batch, float* loss_out,
                                  float* grad_out, int32_t apply, void* ws, size_t ws_bytes,
                                  void* stream);

/* ---------------------------------------------------------------------------
 * Autotuning.  A plan fixes the launch choices of p2m_assemble / p2m_mass_assign /
 * p2m_mass_solve for a shape class: dimension, dtype, field count, and the mesh
 * sides and particles per cell rounded to powers of two.  Plans live in the
 * context (applied while P2M_OPT_PLANS is 1) and can be saved to and loaded from
 * a JSON file.
 * --------------------------------------------------------------------------- */
typedef struct {
    int32_t solver;        /* P2M_SOLVER_* */
    int32_t groups;        /* workgroups of the tile-streaming solve (0: one per compute unit) */
    int32_t scatter_tile;  /* 2D scatter node tile: 0 = default (15 x 15 where it fits), 8 = 8 x 8 */
    int32_t reserved;      /* 0 */
    double inner_rtol;     /* replaces opts->inner_rtol when >= 0 (the inner / outer schedule;
                              the FP64 stopping test on tol is unchanged); < 0: keep opts */
    double time_ms;        /* measured time of one p2m_mass_assign with this plan when tuned */
} p2m_plan;

/* Times p2m_mass_assign of this problem under every applicable plan (each solve
 * kernel; the tile-streaming kernel with one and with half a workgroup per
 * compute unit; the default and the 8 x 8 scatter tile; the caller's inner_rtol,
 * 3e-5, 1e-5, 1e-6 and 0), three runs each after a warm-up, on `stream`; keeps the
 * fastest plan whose solve converged for the problem's shape class and returns it.
 * Synchronises `stream`.  opts->start must
 * be FLIP or ZERO; nodal_out and rep receive the chosen plan's result. */
p2m_status p2m_tune(void* ctx, const p2m_problem* prob, const void* values, int32_t nfields,
                    const p2m_solve_opts* opts, void* nodal_out, p2m_report* rep, void* ws,
                    size_t ws_bytes, void* stream, p2m_plan* best);

/* Batch granularity of the tuner: times p2m_mass_assign_batched of this batch with
 * the caller's inner_rtol, 3e-5, 1e-5, 1e-6 and 0 (one graph build and three timed
 * launches each, on `stream`); keeps the fastest plan under which every instance
 * converged for the batch's shape class (field count, and the instance count, total
 * nodes and total particles rounded to powers of two) and returns it (solver
 * P2M_SOLVER_TILES, groups 0, scatter_tile 0: only inner_rtol applies to a batch).
 * While P2M_OPT_PLANS is 1, p2m_mass_assign_batched takes the inner_rtol of the
 * stored plan of its batch's class; each instance then equals p2m_mass_assign with
 * that inner_rtol bit for bit.  Synchronises `stream`.  opts->start must be FLIP or
 * ZERO; nodal_inout and reps receive the chosen plan's result; P2M_ERR_UNSUPPORTED
 * when no candidate converged. */
p2m_status p2m_tune_batched(void* ctx, const p2m_problem* probs, int32_t nprob,
                            const void* const* values, int32_t nfields, const p2m_solve_opts* opts,
                            void* const* nodal_inout, p2m_report* reps, void* ws, size_t ws_bytes,
                            void* stream, p2m_plan* best);

/* The stored plan of this problem's shape class (P2M_ERR_UNSUPPORTED: none). */
p2m_status p2m_plan_get(void* ctx, const p2m_problem* prob, int32_t nfields, p2m_plan* plan);

/* The stored plan of this batch's shape class (P2M_ERR_UNSUPPORTED: none, or a batch
 * p2m_mass_assign_batched does not take). */
p2m_status p2m_plan_get_batched(void* ctx, const p2m_problem* probs, int32_t nprob,
                                int32_t nfields, p2m_plan* plan);

/* Write every stored plan to `path` (JSON object: shape class -> plan); read
 * plans from such a file into the context (entries of the file replace stored
 * ones of the same class; P2M_ERR_INVALID_ARG for a malformed file, then nothing
 * is loaded); forget every stored plan. */
p2m_status p2m_plan_save(void* ctx, const char* path);
p2m_status p2m_plan_load(void* ctx, const char* path);
p2m_status p2m_plan_clear(void* ctx);

#ifdef __cplusplus
}
#endif

#endif /* P2M_H */

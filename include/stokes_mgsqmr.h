/*
 * stokes_mgsqmr.h - C ABI of the MI355X (gfx950) multigrid-preconditioned SQMR
 * solver for the 3D Stokes equations on a staggered (MAC) grid.
 *
 * Method: Tao & Sifakis, "A Symmetric Multigrid-Preconditioned Krylov Subspace
 * Solver for Stokes Equations" (arXiv 2312.10615).  The library solves
 *
 *     L x = b,   L = [[A, B^T], [B, 0]],  x = (u, p),  b = (f, g)       (Eq. 2)
 *
 * with A = -eta * 7-point Laplacian on each velocity lattice, B^T the pressure
 * gradient onto faces and B minus the divergence onto cells, by SQMR (Alg. 4)
 * preconditioned with one V-cycle (Alg. 1) on the penalised matrix
 * L~ = [[A, B^T], [B, -gamma I]] (Section 4).  The V-cycle smooths with
 * symmetric multiplicative Vanka on the boundary set V1 and symmetric
 * distributive Gauss-Seidel on the interior set V2 (Alg. 3, Section 3),
 * transfers with bilinear / constant prolongation P and R = P^T/8
 * (Section 2), and solves the coarsest level exactly.
 *
 * Domain: a box of nx*ny*nz cells of edge h surrounded by one layer of
 * Dirichlet cells (Section 5 with every cell interior); homogeneous no-slip
 * walls.  Non-zero Dirichlet data is folded into b by the caller.
 *
 * Conventions
 *  - Every function returns an int status (STOKES_OK = 0).  No exception or
 *    abort crosses the ABI.  stokes_strerror() names a status.
 *  - All device pointers are HIP device addresses on the current device;
 *    every GPU operation is enqueued on the stream given to stokes_setup().
 *  - The library never allocates device memory: the caller owns the
 *    workspace, every state vector, and the memory behind them.  The library
 *    allocates only its host-side context, released by stokes_destroy().
 *  - One context must not be used from two host threads at once.
 *
 * State vectors ("x", "b", "s", "t", "y" below) are float64 device arrays of
 * stokes_layout_t.total elements holding u_x, u_y, u_z and p in the padded
 * layout described by stokes_layout(): padded cell (I, J, K), I in [0, nx+2),
 * J in [0, ny+2), K in [0, nz+2), is slot s = I + sy*J + sz*K, and field f of
 * slot s is element off[f] + (s & 1) * (field / 2) + (s >> 1) (the red/black
 * split, see stokes_layout_t).  Pressure of cell (i,j,k) (0-based) is at (i+1, j+1, k+1);
 * u_x on the face x = i*h of row (j,k) is at (i+1, j+1, k+1), i = 0..nx
 * (i = 0 and i = nx are walls); u_y, u_z alike.  Slots that are not unknowns
 * ("ghost slots": walls, Dirichlet ghosts, pitch padding) must hold zero in
 * every input that the library reads as x; the library writes zero there in
 * every vector it outputs.  Right-hand sides may hold anything in ghost slots.
 * A field also has elements that are no slot (its spare tail, and the one
 * element between two planes when sy*(ny+2) is even): they are zero in the x
 * of stokes_solve and the t of stokes_vcycle, never read as input, and left
 * as they are in the other outputs.
 */
#ifndef STOKES_MGSQMR_H
#define STOKES_MGSQMR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  STOKES_OK = 0,
  STOKES_EINVAL = 1,      /* bad dimensions / levels / null or misaligned pointer / small workspace */
  STOKES_ENOCONV = 2,     /* maxit reached before the tolerance; x holds the last iterate */
  STOKES_EBREAKDOWN = 3,  /* sigma = 0 or rho = 0 in SQMR; x holds the last iterate */
  STOKES_ENONFINITE = 4,  /* a NaN/Inf scalar appeared (e.g. non-finite b) */
  STOKES_EDEVICE = 5,     /* a HIP runtime call failed */
  STOKES_ETOOLARGE = 6    /* stokes_solve_static: the workspace would exceed STOKES_STATIC_BYTES */
};

/* Smoothing schedules of the V-cycle (Section 3: the pre- and post-smoothing
 * matrices must be transposes of each other for W to be symmetric).
 *  STOKES_SMOOTHER_SYMMETRIC: the paper's arrangement - the same symmetric
 *    smoother (Alg. 3 with one symmetric DGS = forward + reverse sweep) in both
 *    phases, nu/2 times (nu even).  Default.
 *  STOKES_SMOOTHER_SPLIT: pre-smoothing = Alg. 3 with nu reverse DGS sweeps
 *    (Gauss-Seidel on M^T L~, Eq. ldist) on V2 between symmetric Vanka on V1;
 *    post-smoothing = Alg. 3 with nu forward DGS sweeps (on L~ M, Eq. dist).
 *    The two are transposes of each other.
 * Every DGS sweep takes the velocities red, black (lattice parity) and the
 * pressures by the eight colour classes (i&1) + 2(j&1) + 4(k&1), 0..7 forward
 * and 7..0 in the reverse sweep. */
enum { STOKES_SMOOTHER_SPLIT = 0, STOKES_SMOOTHER_SYMMETRIC = 1 };

/* The V1 (boundary) smoother of Alg. 3 (Section 3.2):
 *  STOKES_VANKA_MULT8: symmetric multiplicative Vanka, the paper's 8 colour
 *    classes (i&1) + 2(j&1) + 4(k&1) in the order 0 7 1 6 2 5 3 4 and then
 *    the reverse (the paper fixes no order of the classes; here each class is
 *    followed by its complement), each class updated at once from the state
 *    at its start.  Complementary classes share no unknown and read none of
 *    each other's, so each pair runs as one pass with the same values.
 *    Default.
 *  STOKES_VANKA_MULT27: the same with 27 classes (i%3) + 3(j%3) + 9(k%3);
 *    same-class cells are three apart and share no stencil entry, so a class
 *    step equals solving its subdomains one after another (Eq. mv).
 *  STOKES_VANKA_ADDITIVE: additive Vanka (Eq. av), every V1 subdomain from
 *    the same residual, corrections summed (applied class by class so that
 *    shared faces are summed in a fixed order); symmetric by itself. */
enum { STOKES_VANKA_MULT8 = 0, STOKES_VANKA_MULT27 = 1, STOKES_VANKA_ADDITIVE = 2 };

/* Solver parameters.  Defaults (stokes_default_params): eta = 1, gamma = 1e-3
 * (the penalty of Section 4; Section 6 uses 1e-3), levels = 0 (auto), nu = 2,
 * n_boundary = 1, vcycle_precision = 64, smoother = STOKES_SMOOTHER_SYMMETRIC,
 * flags = STOKES_FLAG_REMOVE_MEAN, vanka = STOKES_VANKA_MULT8, cycle = 1. */
typedef struct stokes_params {
  int32_t nx, ny, nz;         /* interior cells per axis, each >= 2 */
  double h;                   /* cell edge; > 0 */
  double eta;                 /* viscosity; > 0 */
  double gamma;               /* penalty of L~ inside the V-cycle; > 0 (with 0 the coarsest L~ of a
                                 closed box is singular: constant pressure is in its null space) */
  int32_t levels;             /* multigrid levels; 0 = halve while all axes are even and
                                 every halved axis keeps >= 4 cells; explicit values may
                                 go down to 2 cells per axis */
  int32_t nu;                 /* DGS sweeps per smoothing phase (pre and post), >= 1;
                                 even for STOKES_SMOOTHER_SYMMETRIC */
  int32_t n_boundary;         /* symmetric Vanka applications per Vanka slot of Alg. 3, >= 1 */
  int32_t vcycle_precision;   /* 64: FP64 V-cycle.  32: the V-cycle's level vectors, smoother,
                                 transfer and stencil arithmetic in FP32 (s converted on entry,
                                 t converted back on exit, coarsest solve accumulated in FP64);
                                 SQMR recurrences, inner products and the true residual stay FP64 */
  int32_t smoother;           /* STOKES_SMOOTHER_* */
  int32_t flags;              /* STOKES_FLAG_* */
  int32_t vanka;              /* STOKES_VANKA_* */
  int32_t cycle;              /* 1: V-cycle (Alg. 1).  2: W-cycle - the coarse correction of every
                                 level above the coarsest is two cycles of the next level, the
                                 second starting from the first's result (Section 2) */
  const uint8_t* labels;      /* NULL: the box of nx*ny*nz interior cells padded by Dirichlet cells.
                                 Else host cell labels of Section 5 for the padded box, one byte per
                                 cell, x fastest ((nx+2)(ny+2)(nz+2) bytes): 0 interior, 1 Dirichlet,
                                 2 exterior; the outer layer holds no interior cell.  Read during
                                 stokes_workspace_bytes / stokes_setup only (the caller keeps
                                 ownership).  Faces of Dirichlet cells hold Dirichlet values; a face
                                 with an interior cell beside it and no Dirichlet cell is an unknown
                                 (between an interior and an exterior cell it carries the Neumann
                                 condition: zero exterior pressure, zero normal derivative of the
                                 velocity); V1 = interior cells within one cell (face, edge or
                                 corner) of a Dirichlet cell or two of an exterior cell.  Coarse
                                 labels follow Section 5.  Single-box solver only (the batch calls
                                 reject labels).  With an exterior cell beside an unknown face the
                                 pressure is unique and STOKES_FLAG_REMOVE_MEAN does nothing. */
} stokes_params;

/* After convergence subtract the mean pressure over the cells (the closed box
 * leaves p defined up to a constant). */
#define STOKES_FLAG_REMOVE_MEAN 1
/* Launch the V-cycle kernel by kernel instead of replaying a captured HIP
 * graph of it (the default captures one graph per (s, t) pointer pair and
 * profiling selection, on a private stream, and replays it on the caller's
 * stream). */
#define STOKES_FLAG_NO_GRAPH 2

/* A state vector holds u_x, u_y, u_z, p, each over the padded slots
 * s = I + sy J + sz K (I in [0, nx+1], ... ; cell (I,J,K) owns p(I,J,K) and
 * its minus faces u_x(I,J,K), u_y(I,J,K), u_z(I,J,K)).  sy and sz are odd, so
 * s & 1 is the red/black colour of the slot, and each field stores its two
 * colours apart: field f's slot s is element
 *     off[f] + (s & 1) * (field / 2) + (s >> 1).
 * Elements that are not unknowns hold 0. */
typedef struct stokes_layout_t {
  int32_t nx, ny, nz;         /* interior cells */
  int64_t sy, sz;             /* slot pitches of J and K (odd; the pitch of I is 1) */
  int64_t off[4];             /* element offset of u_x, u_y, u_z, p */
  int64_t field;              /* elements per field (off[f+1] - off[f]), a multiple of 8 */
  int64_t total;              /* elements in one state vector */
  int64_t n_dofs;             /* number of unknowns */
  int32_t levels;             /* resolved level count */
} stokes_layout_t;

typedef struct stokes_info {
  int32_t iters;              /* SQMR iterations performed */
  int32_t status;             /* STOKES_OK / ENOCONV / EBREAKDOWN / ENONFINITE */
  double relres;              /* final true ||b - L x||_2 / ||b||_2 */
  double bnorm;               /* ||b||_2 over the unknowns */
  double* history;            /* optional caller-owned host array of maxit+1 doubles:
                                 relative true residual after each iteration (index 0: x0);
                                 NULL = not recorded */
} stokes_info;

typedef struct stokes_ctx stokes_ctx;

/* Fill *p with the defaults listed above and the given box. */
int stokes_default_params(int32_t nx, int32_t ny, int32_t nz, double h, stokes_params* p);

/* Bytes of device workspace stokes_setup() needs for these parameters. */
int stokes_workspace_bytes(const stokes_params* p, size_t* bytes);

/* Build the multigrid hierarchy (label coarsening of Section 5, rediscretised
 * operators of Section 2), the Vanka local inverses (the prefactorised local
 * saddle problems of Section 6), the coarsest-level inverse and the V1 colour
 * lists, and upload them into `workspace` (device, >= stokes_workspace_bytes,
 * 256-byte aligned).  `hip_stream` is a hipStream_t (NULL = default stream).
 * Blocks until the uploads are complete.  On success *out owns a host context. */
int stokes_setup(const stokes_params* p, void* workspace, size_t bytes, void* hip_stream,
                 stokes_ctx** out);

/* Layout of state vectors for this context. */
int stokes_layout(const stokes_ctx* ctx, stokes_layout_t* out);

/* Layout of the state vectors of multigrid level `level` (0 = finest, up to
 * levels - 1): the same padded layout for the level's box of cells; `levels`
 * reports the number of levels from this one down. */
int stokes_level_layout(const stokes_ctx* ctx, int32_t level, stokes_layout_t* out);

/* Grid transfers between the finest level and the next (Section 2): coarse =
 * R fine with R = P^T / 8, and fine = P coarse (fine is overwritten), P the
 * prolongation of the V-cycle (trilinear per staggered lattice, constant for
 * p).  fine uses the level-0 layout, coarse the level-1 layout; inputs must be
 * zero at slots that are not unknowns, outputs are.  FP64, async on the
 * context's stream.  EINVAL for a one-level context or aliased vectors.
 * Used to carry a warm start computed on the coarser grid to the finest one. */
int stokes_restrict(stokes_ctx* ctx, const double* fine, double* coarse);
int stokes_prolong(stokes_ctx* ctx, const double* coarse, double* fine);

/* Dirichlet data moved to the right-hand side (Section 5): out = b - L g at
 * the unknowns and 0 elsewhere, where g is a state vector that holds the
 * boundary values in its slots that are not unknowns (tangential velocities
 * in the ghost slots of the Dirichlet cells, wall-normal velocities on the
 * wall faces) and 0 at the unknowns.  The solution of L x = out plus g is the
 * discrete solution with those boundary values (e.g. the lid of the driven
 * cavity of Section 6).  Async; out must differ from g and b. */
int stokes_lift(stokes_ctx* ctx, const double* g, const double* b, double* out);

/* y = L x (penalized = 0) or y = L~ x (penalized = 1) on the finest level
 * (Eq. 2 / Section 4).  x and y are distinct device state vectors.  Async. */
int stokes_apply(stokes_ctx* ctx, const double* x, double* y, int32_t penalized);

/* t = W s: one V-cycle on L~ with zero initial guess (Alg. 1 as the
 * preconditioner of Section 3/4).  s and t are distinct device state vectors;
 * s is not modified.  Async. */
int stokes_vcycle(stokes_ctx* ctx, const double* s, double* t);

/* Solve L x = b with MG-SQMR (Alg. 4).  b: device state vector (read only).
 * x: device state vector, in: initial guess x0 (zeros or a warm start; its
 * ghost slots are cleared), out: the iterate meeting ||b - L x|| <= rtol ||b||
 * (or the last one).  Stops after maxit iterations (maxit >= 0).  Synchronises
 * the stream (the SQMR scalars are read back every iteration).  Returns the
 * solve status, also stored in info->status (info may be NULL). */
int stokes_solve(stokes_ctx* ctx, const double* b, double* x, double rtol, int32_t maxit,
                 stokes_info* info);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): stokes_solve with no
 * context and no workspace argument.  The set-up, the solve and the tear-down
 * of stokes_setup / stokes_solve / stokes_destroy run on a workspace inside
 * the library, a device array of STOKES_STATIC_BYTES (one per GPU, held until
 * the process ends); the call makes no device or pinned-host allocation and
 * creates no stream, event or graph (its V-cycles launch kernel by kernel).
 * p, b, x, rtol, maxit and info as for stokes_setup and stokes_solve; work
 * goes on hip_stream (the current device's), and the call returns after the
 * stream completes.  STOKES_ETOOLARGE when stokes_workspace_bytes(p) exceeds
 * STOKES_STATIC_BYTES (64 MiB: boxes up to 64^3 cells), before any GPU work.
 * Every call on one GPU uses the same array and leaves its contents behind
 * (the set-up clears what must start at zero): calls that overlap on one GPU
 * (two host threads, or two streams) race and must not be issued. */
#define STOKES_STATIC_BYTES (64u << 20)
int stokes_solve_static(const stokes_params* p, const double* b, double* x, double rtol, int32_t maxit,
                        stokes_info* info, void* hip_stream);

/* Diagnostics: per-kernel timing with HIP events recorded on the context's
 * stream around the selected launches (the "tracing" aux subsystem).
 * kernel_class: one of STOKES_KC_*, or STOKES_KC_ALL, or STOKES_KC_OFF to stop;
 * level: multigrid level (0 = finest) or -1 for all.  Selecting resets the
 * accumulated times.  stokes_profile_read() synchronises the stream and returns
 * the accumulated milliseconds and launch count for (kernel_class, level). */
enum {
  STOKES_KC_APPLY = 0,        /* operator / residual / residual-norm passes */
  STOKES_KC_DGS_U = 1,        /* velocity Gauss-Seidel half sweep (one colour) */
  STOKES_KC_DGS_PF_OWN = 2,   /* forward pressure launches 0..3: own steps of one stage of pressure
                                 classes, with the previous stage's neighbour updates */
  STOKES_KC_DGS_PF_NBR = 3,   /* forward pressure launch 4: the last stage's neighbour updates */
  STOKES_KC_DGS_PR = 4,       /* reverse (left-preconditioned) pressure step, one stage */
  STOKES_KC_VANKA_DELTA = 5,  /* Vanka local solves of one colour (with their corrections on levels that
                                 keep two copies of the state; a whole Vanka step on small levels) */
  STOKES_KC_VANKA_APPLY = 6,  /* Vanka corrections of one colour, or the second copy's band update */
  STOKES_KC_RESTRICT = 7,
  STOKES_KC_PROLONG = 8,
  STOKES_KC_COARSE = 9,
  STOKES_KC_BLAS = 10,        /* SQMR vector updates, dots, fills */
  STOKES_KC_COUNT = 11,
  STOKES_KC_ALL = -1,
  STOKES_KC_OFF = -2
};
int stokes_profile(stokes_ctx* ctx, int32_t kernel_class, int32_t level);
int stokes_profile_read(stokes_ctx* ctx, int32_t kernel_class, int32_t level, double* total_ms, int64_t* launches);

/* Release the host context (never touches the caller's device memory). */
void stokes_destroy(stokes_ctx* ctx);

/* ------------------------------------------------------------------ batches
 * Many independent boxes solved together with MG-SQMR (the same method and
 * schedule per box as stokes_solve).  Every kernel launch covers one step of
 * the method for all boxes that take part in it, the SQMR scalars of every
 * box stay on the device, a box that has finished drops out of later
 * launches, and the iterations run as replays of captured HIP graphs (the
 * first one holds the set-up phase and the first `first` iterations, each
 * later one `later` iterations; defaults 10 and 2).
 *
 * p[0..n) gives each box its own size, spacing and levels (levels = 0: the
 * single-box automatic rule, deepened while the coarsest system would exceed
 * 2500 unknowns); nu, n_boundary, smoother and vcycle_precision must be equal
 * for all boxes, vanka must be STOKES_VANKA_MULT8 and cycle 1.  Box d's state vector is the slice [offset_d, offset_d +
 * total_d) of one batch vector of stokes_batch_size() doubles
 * (stokes_batch_layout); slots between slices are ignored.
 * Ownership, streams and statuses as for a single box; the library allocates
 * only its host context and two small pinned host buffers. */
typedef struct stokes_batch stokes_batch;

int stokes_batch_workspace_bytes(int32_t n, const stokes_params* p, size_t* bytes);
int stokes_batch_setup(int32_t n, const stokes_params* p, void* workspace, size_t bytes, void* hip_stream,
                       stokes_batch** out);
int stokes_batch_layout(const stokes_batch* batch, int32_t box, int64_t* offset, stokes_layout_t* out);
int stokes_batch_size(const stokes_batch* batch, int64_t* total);

/* Tile shapes of the stencil kernels (x-extent of a block's 2-D tile: 32, 64,
 * 128 or 256 items): times every shape of every kernel class on every level
 * of this batch and keeps the fastest.  Synchronises.  choices (optional,
 * host int[8 * 16]) receives the x-extent per [class][level] (0 = unused). */
int stokes_batch_autotune(stokes_batch* batch, int32_t* choices);

/* Iterations per graph replay (first >= 0, later >= 1). */
int stokes_batch_set_chunks(stokes_batch* batch, int32_t first, int32_t later);

/* Solve every box: b, x batch vectors (x in: initial guesses, out: iterates),
 * rtol and maxit as for stokes_solve; info: host array of n entries (history
 * is not recorded).  Synchronises.  Returns STOKES_OK when every box
 * converged, else the status of the first box that did not. */
int stokes_batch_solve(stokes_batch* batch, const double* b, double* x, double rtol, int32_t maxit,
                       stokes_info* info);

void stokes_batch_destroy(stokes_batch* batch);

const char* stokes_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* STOKES_MGSQMR_H */

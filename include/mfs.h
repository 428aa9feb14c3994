/*
 * mfs.h -- C ABI of the MI355X (gfx950) mixed-FEM skinning solver.
 *
 * The library computes, for one rig pose, the deformed vertex positions of a
 * tetrahedral character mesh by the mixed finite element method of "Automatic
 * Skinning using the Mixed Finite Element Method" (Song et al.): per-element
 * symmetric stretches S_k are tied to the vertex positions through rotations
 * R_k fixed by the rig (Section 3, the mixed form and its constraint), vertices
 * near the skeleton are pinned with a quadratic penalty whose targets follow
 * their handle (Section 3, the constraint C(x); Section 3.2, "Initial shape
 * preservation"), and the multipliers and stretches are condensed into a
 * vertex-only symmetric positive definite system (Section 3, the condensed
 * per-vertex system and the pseudo-inverse of [R]).  One frame is one pass of
 * the loop of Algorithm 1: the rig pose sets [R], the system is assembled and
 * solved.  For quadratic energies (ARAP, co-rotated linear) one solve is the
 * optimum; for neo-Hookean the frame runs Newton iterations.
 *
 * Conventions (all entry points):
 *   - Every call returns int: 0 = MFS_OK, > 0 = warning, < 0 = error.  The
 *     text of the last error on the calling thread is mfs_last_error().
 *   - Inputs are read during the call only; the library never keeps caller
 *     pointers.  Output buffers are allocated by the caller.
 *   - Pointers marked "host or device" follow the call's memory-space field:
 *     MFS_MEM_HOST = ordinary host memory, MFS_MEM_DEVICE = device memory of
 *     the context's GPU.
 *   - Opaque handles are owned by the library and released by *_destroy.
 *   - A context and everything made from it are used by one host thread at a
 *     time.  All GPU work is enqueued on the context's stream; calls that
 *     return results to the host synchronise that stream.
 *   - Arrays are row-major; vertex positions are n x 3 doubles, rotations
 *     are 3 x 3 row-major (9 doubles) mapping rest to posed space.
 */
#ifndef MFS_H
#define MFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define MFS_OK 0
#define MFS_W_NOT_CONVERGED 1   /* best iterate written; see mfs_solve_stats */
#define MFS_E_INVALID (-1)      /* bad argument: index out of range, non-finite value,
                                   nu outside (-1, 0.5), E <= 0, non-rotation handle */
#define MFS_E_DEGENERATE (-2)   /* rest tet with |det Dm| <= 1e-12 * (mean edge)^3 */
#define MFS_E_SINGULAR (-3)     /* pins cannot remove rigid motion (< 3 non-collinear) */
#define MFS_E_OOM (-4)          /* device allocation failed */
#define MFS_E_HIP (-5)          /* HIP runtime error */
#define MFS_E_BUSY (-6)         /* serving queue full / workspace budget exhausted */
#define MFS_E_UNSUPPORTED (-7)  /* option combination not implemented */

/* ---- enumerations ---------------------------------------------------- */
enum mfs_material {        /* per-element stretch energy Psi(S) */
  MFS_ARAP = 0,            /* mu ||S - I||^2 */
  MFS_COROT = 1,           /* mu ||S - I||^2 + lambda/2 tr(S - I)^2 */
  MFS_NEOHOOKEAN = 2       /* mu/2 (tr(S S) - 3) - mu ln J + lambda/2 (ln J)^2, J = det S */
};
enum mfs_precision {
  MFS_FP64 = 0,            /* every kernel in FP64 */
  MFS_FP32_REFINED = 1     /* FP32 Hessian values and PCG; FP64 positions, stretches,
                              gradient (residual), energies and updates */
};
enum mfs_memory { MFS_MEM_HOST = 0, MFS_MEM_DEVICE = 1 };
enum mfs_warm_start {
  MFS_WARM_REST = 0,       /* x0 = rest positions (Algorithm 1, x <- X) */
  MFS_WARM_PREVIOUS = 1    /* x0 = this character's last solved positions */
};

typedef struct mfs_context mfs_context;
typedef struct mfs_character mfs_character;

/* ---- descriptors ----------------------------------------------------- */
typedef struct mfs_mesh_desc {
  int64_t n_vertices;              /* n >= 4 */
  const double* rest_positions;    /* n x 3 rest positions X */
  int64_t n_tets;                  /* m >= 1 */
  const int32_t* tets;             /* m x 4 vertex indices (any orientation) */
  const int32_t* material_model;   /* m, enum mfs_material */
  const double* youngs;            /* m, Young's modulus E > 0 */
  const double* poisson;           /* m, Poisson ratio in (-1, 0.5) */
  int32_t n_handles;               /* rig handles, 1..256 */
  const int32_t* tet_cluster;      /* m, handle whose rotation the tet takes */
  int64_t n_pins;                  /* >= 3 */
  const int32_t* pin_vertex;       /* n_pins vertex indices (repeats allowed) */
  const int32_t* pin_handle;       /* n_pins handle indices */
  double pin_stiffness;            /* k_s > 0 */
  int32_t memory_space;            /* enum mfs_memory of the arrays above */
} mfs_mesh_desc;

typedef struct mfs_solve_opts {
  int32_t precision;        /* enum mfs_precision */
  int32_t max_newton;       /* iteration cap (the first, mixed step counts) */
  int32_t fixed_newton;     /* 1: run exactly max_newton iterations */
  double step_tol;          /* stop when max_v ||alpha dx_v|| <= step_tol * bbox diagonal
                               in a Newton-phase iteration */
  double cg_tol;            /* PCG stop: ||r|| <= cg_tol ||b|| */
  int32_t cg_max;           /* PCG iteration cap per solve */
  int32_t warm_start;       /* enum mfs_warm_start */
  int32_t output_memory;    /* enum mfs_memory of x_out */
  int32_t cg_adaptive;      /* 1: inexact Newton: once s = J x, each PCG solve stops at
                               max(cg_tol, eta_k) with the Eisenstat-Walker forcing
                               eta_k = min(0.1, 0.9 (|g_k| / |g_k-1|)^2); mixed-phase
                               solves keep cg_tol */
  int32_t load_bisections;  /* robustness for large poses (0: off): when the mixed phase
                               stalls (more than 6 mixed steps, or no feasible step),
                               return to the last converged state and approach the pose
                               through intermediate poses -- each handle's screw motion
                               T(tau) = T0 exp(tau log(T0^-1 T1)) in SE(3) from the
                               warm-start pose T0 to the target T1 -- halving the increment
                               at most this many times and doubling it after each
                               intermediate pose converges (to a 1e-4 * bbox step) */
  int32_t fp32_cg_max;      /* FP32_REFINED: a Newton step whose FP32 PCG has not converged
                               after this many iterations (or broke down) is solved again in
                               FP64 (element records, assembly, and a PCG started from the
                               FP32 iterate); 0 = 100 n^(1/3), at least 8000 */
} mfs_solve_opts;

typedef struct mfs_solve_stats {
  int32_t status;           /* return code of the solve */
  int32_t iterations;       /* Newton iterations run, mixed steps included */
  int32_t mixed_iterations; /* steps taken while s != J x */
  int32_t cg_iterations;    /* PCG iterations summed over the frame */
  int32_t halvings;         /* line-search halvings summed over the frame */
  int32_t clamped;          /* neo-Hookean elements with clamped Hessian, last iteration */
  int32_t fp64_routed;      /* tets whose polar decomposition ran in FP64 (FP32 path) */
  int32_t cg_not_converged; /* solves that hit cg_max (or stopped by a breakdown) */
  double energy;            /* E(x) at the returned positions */
  double grad_norm;         /* ||grad E|| at the last Newton-phase assembly */
  double last_step;         /* max_v ||alpha dx_v|| of the last iteration */
  double cg_rel_residual;   /* ||r|| / ||b|| of the last PCG solve */
  int32_t fp64_resolves;    /* FP32_REFINED: Newton steps re-solved in FP64 (fp32_cg_max) */
  int32_t fp64_resolve_cg_iterations; /* PCG iterations of those re-solves (included in cg_iterations) */
} mfs_solve_stats;

/* ---- library and context --------------------------------------------- */

/* Fill *opts with the defaults: FP64, max_newton 50, fixed_newton 0,
 * step_tol 1e-10, cg_tol 1e-10, cg_max 20000, warm start REST, host output,
 * fixed PCG tolerance (cg_adaptive 0), load_bisections 6 (ignored when
 * fixed_newton is set). */
void mfs_default_opts(mfs_solve_opts* opts);

/* Text for a status code (static storage). */
const char* mfs_status_string(int status);

/* Text of the last error reported on the calling thread ("" if none). */
const char* mfs_last_error(void);

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * (e.g. the caller's current stream) or NULL for a stream owned by the
 * context.  Every kernel and copy of this context is enqueued on it. */
int mfs_context_create(int device, void* hip_stream, mfs_context** out);
int mfs_context_destroy(mfs_context* ctx);

/* Launch-shape knobs of a context (set by the autotuner or by hand). */
typedef struct mfs_tuning {
  int32_t pcg_lanes_per_row;  /* lanes per block row in the PCG SpMV: 2, 4 or 8 */
  int32_t use_graphs;         /* 1: replay runs of PCG iterations as captured HIP graphs */
  int32_t graph_iterations;   /* PCG iterations per captured graph, 1..64 */
  int32_t first_check;        /* PCG iterations in the first queued chunk of a solve */
  int32_t min_run, max_run;   /* later chunks: min_run iterations (at most max_run).  Chunks are
                                 queued one ahead of the running one; the kernels raise a
                                 host-mapped flag when a system stops, so the host never
                                 synchronises to check convergence */
  int32_t pcg_pipelined;      /* 1: solves run the pipelined PCG of Ghysels and Vanroose (one
                                 kernel per iteration, dot products overlapped with the SpMV;
                                 FP64 vectors and recurrences, the matrix in the solve's
                                 precision).  The FP64 re-solves inside an FP32_REFINED solve
                                 always run the two-kernel form */
  int32_t allread_max_tiles;  /* PCG dot products of a system with at most this many 64-row
                                 tiles are folded by every workgroup of the next kernel
                                 (no fences); larger systems fold them in the last workgroup
                                 to finish (arrival ticket with a release fence) */
  int32_t pcg_persistent;     /* 1 (FP32_REFINED solves): a pipelined PCG whose workgroups
                                 (one per 64-row tile of every system in the batch, the
                                 tile's matrix rows held in LDS) all fit on the device at
                                 once runs as one cooperative launch with a barrier per
                                 iteration instead of one launch per iteration; the
                                 iterates are the same bitwise.  Default 0: it pays off for
                                 small systems, where the launch per iteration dominates
                                 (the autotuner tries it) */
  int32_t batch_async;        /* 1 (default): a batch of two or more characters
                                 (mfs_solve_batch) whose solves run the two-kernel or the
                                 pipelined PCG (not the persistent launch) lets each
                                 character run its own Newton steps: a character whose PCG
                                 solve has stopped takes its line search, update and next
                                 element pass and assembly while the others' solves go on,
                                 and every PCG launch covers the characters solving at that
                                 moment (launched directly, not as graphs); 0: every
                                 character of the batch runs the same Newton iteration,
                                 which waits for the slowest PCG solve.  A single character
                                 and the server's lanes always run the second form.
                                 Results are the same bitwise either way */
} mfs_tuning;

int mfs_context_get_tuning(const mfs_context* ctx, mfs_tuning* out);
/* Validates every field (MFS_E_INVALID otherwise) and drops cached graphs. */
int mfs_context_set_tuning(mfs_context* ctx, const mfs_tuning* tuning);

/* ---- characters (resident per-mesh state) ----------------------------- */

/* Copy a character to the device and precompute its rest data: the shape
 * gradients Dm^-1 and volumes W_k (Section 3: F = B x and the element
 * volumes of the discrete mixed energy), Lame parameters from (E, nu), the
 * 3x3-block sparsity pattern of the condensed matrix and its
 * element-to-block assembly map, and a bandwidth-reducing vertex order.
 * Errors: MFS_E_INVALID, MFS_E_DEGENERATE, MFS_E_SINGULAR, MFS_E_OOM,
 * MFS_E_HIP.  On error *out is NULL. */
int mfs_character_create(mfs_context* ctx, const mfs_mesh_desc* desc, mfs_character** out);
int mfs_character_destroy(mfs_character* ch);

/* Device bytes that mfs_character_create would allocate for this mesh,
 * computed on the host before anything is uploaded, so that a caller can
 * admit a character, or size a server's arena, by its memory footprint
 * (Algorithm 1's inputs: the rest tet mesh and its pins).  resident_bytes:
 * what the character keeps between frames (mesh data, assembly map,
 * positions and stretches); workspace_bytes: one frame solve's workspace
 * (element state, matrix values, PCG vectors, reductions), the amount a
 * server lends a character whose workspace was released.  Reads n_vertices,
 * n_tets, tets, n_pins and memory_space only (tets host or device); the
 * matrix has one 3x3 block per vertex and two per mesh edge.  No GPU work
 * for host arrays.  Either output may be NULL.  Errors: MFS_E_INVALID
 * (sizes out of range, a vertex index out of range, a tet repeating a
 * vertex, a vertex in no tet: the checks of mfs_character_create on these
 * fields), MFS_E_HIP (device tets). */
int mfs_character_footprint(const mfs_mesh_desc* desc, size_t* resident_bytes,
                            size_t* workspace_bytes);

/* The same two byte counts for a created character, as allocated. */
int mfs_character_get_footprint(const mfs_character* ch, size_t* resident_bytes,
                                size_t* workspace_bytes);

/* External vertex forces (the f_ext term of the next-step extensions: a
 * load b += f_ext on selected vertices, potential -f . x in E), used by
 * every later solve and evaluation of this character until changed.
 * vertices: count indices (repeats add up), forces: count x 3, host or
 * device per memory_space; count = 0 removes all forces.  Synchronises the
 * context's stream.  Errors: MFS_E_INVALID (index out of range, non-finite
 * force), MFS_E_OOM. */
int mfs_character_set_forces(mfs_character* ch, const int32_t* vertices, const double* forces,
                             int64_t count, int32_t memory_space);

/* Free the character's own solve workspace (workspace_bytes of device
 * memory), keeping its resident data and last solution.  A server then
 * lends it a workspace from its arena for each admitted frame; a later
 * standalone call (solve, batch, evaluate) allocates the workspace again.
 * Synchronises the context's stream. */
int mfs_character_release_workspace(mfs_character* ch);

/* ---- rig helpers ------------------------------------------------------ */

/* Rotation clusters (Section 3.1): each tet takes the handle of the bone
 * segment nearest its barycenter; ties go to the lowest segment index, and a
 * zero-length segment is a point handle.  X: n x 3, tets: m x 4, seg_a/seg_b:
 * nseg x 3, seg_handle: nseg, out: m (all host or device per memory_space).
 * Runs on the GPU of ctx; returns after out is written. */
int mfs_cluster_by_segments(mfs_context* ctx, const double* X, int64_t n,
                            const int32_t* tets, int64_t m, int32_t nseg,
                            const double* seg_a, const double* seg_b,
                            const int32_t* seg_handle, int32_t* out, int32_t memory_space);

/* Rotation smoothing across cluster boundaries.  The paper names the
 * rotation discontinuities between clusters as its main limitation and
 * leaves smoothing to future work (Section 5, Limitations; Section 4,
 * rotation clustering); this is one reading of it.  Per tet, with d the
 * distance from the barycenter to a bone segment (as in
 * mfs_cluster_by_segments) and a handle's distance that of its nearest
 * segment: the handle of the nearest segment first, weight 1; then the other
 * handles h with d_h < d_min + width, weight 1 - (d_h - d_min) / width, in
 * decreasing weight (ties: lower handle index first); at most kmax (1..4) in
 * all, the weights divided by their sum.  Unused entries: handle -1, weight
 * 0.  out_handles, out_weights: m x kmax row-major.  width = 0 reproduces
 * the clusters.  All arrays host or device per memory_space; returns after
 * the outputs are written. */
int mfs_blend_weights(mfs_context* ctx, const double* X, int64_t n, const int32_t* tets, int64_t m,
                      int32_t nseg, const double* seg_a, const double* seg_b, const int32_t* seg_handle,
                      int32_t n_handles, double width, int32_t kmax, int32_t* out_handles,
                      double* out_weights, int32_t memory_space);

/* Smoothed tet rotations for later solves, evaluations and stress
 * recovery: for every pose, R_k = the rotation factor of the polar
 * decomposition of sum_j w_kj R_{h_kj} (the handle rotation itself for a
 * tet with one handle, or where the blend has det <= 0) replaces the
 * rotation of the tet's cluster.  handles, weights: m x kmax row-major in
 * the caller's tet order (e.g. from mfs_blend_weights); the first handle of
 * every tet must be valid, -1 marks unused entries, weights finite and >= 0
 * (their scale does not matter).  handles = NULL returns to cluster
 * rotations.  Synchronises the context's stream; not while a frame of the
 * character is in flight.  Pins keep following their handles. */
int mfs_character_set_rotation_blend(mfs_character* ch, int32_t kmax, const int32_t* handles,
                                     const double* weights, int32_t memory_space);

/* ---- solving ------------------------------------------------------------ */

/* Solve one frame (Algorithm 1, one pose).  handle_R: n_handles x 9 and
 * handle_t: n_handles x 3 on the host give each handle's rest->posed rigid
 * transform; a tet in cluster h takes rotation R_h, and a pin on handle h
 * targets R_h X_p + t_h.  x_out: n x 3 in the caller's vertex order, host or
 * device per opts->output_memory.  stats may be NULL.  A rotation with
 * ||R^T R - I|| > 1e-9 or det R <= 0 is MFS_E_INVALID.  Returns MFS_OK, or
 * MFS_W_NOT_CONVERGED with the best iterate written when the line search
 * fails or the iteration cap is hit before the step tolerance. */
int mfs_solve_frame(mfs_character* ch, const double* handle_R, const double* handle_t,
                    const mfs_solve_opts* opts, double* x_out, mfs_solve_stats* stats);

/* Solve one frame for each of `count` characters of one context together:
 * every kernel launch covers the tiles of all characters still iterating,
 * with per-character scalars, convergence flags and reductions, so each
 * character's result is the same as when it is solved alone.  R[i], t[i],
 * x_out[i] as in mfs_solve_frame; stats: count entries or NULL.  Returns the
 * most severe status over the batch. */
int mfs_solve_batch(mfs_context* ctx, int32_t count, mfs_character* const* chars,
                    const double* const* handle_R, const double* const* handle_t,
                    const mfs_solve_opts* opts, double* const* x_out,
                    mfs_solve_stats* stats);

/* ---- autotuning --------------------------------------------------------- */

#define MFS_AUTOTUNE_FORCE 1  /* time the candidates even when a cached choice exists */

/* Choose the PCG launch schedule (PCG form: two-kernel, pipelined, or
 * pipelined in one persistent launch; SpMV lanes per row, PCG iterations per
 * graph, first convergence check, shortest run between checks) for a batch
 * like this one and apply it to the context.  Each candidate solves the
 * given frames (as mfs_solve_batch with `opts`, but from the rest shape and
 * for exactly `newton_iterations` iterations, or, with newton_iterations 0,
 * as whole frames under `opts`' stop rule and Newton cap, into scratch
 * device memory) twice, timing the second.  A batch in the asynchronous
 * form is timed at one graph length only (it launches directly).  A candidate's time is scaled by the default
 * schedule's total PCG iteration count over its own (summation order alone
 * moves the counts by a few percent), and the winner is the fastest
 * candidate by that time whose solves are as good as the default
 * schedule's: no PCG solve left
 * unconverged (or stopped by a breakdown) where the default had none, and
 * every final gradient norm within 10x the default's.  Choices are kept per
 * (GPU architecture, size class = bit length of the total vertex count):
 * in the context, and in the text file `cache_path` when it is not NULL
 * (read first, rewritten after tuning).  A cached choice is applied without
 * timing unless flags has MFS_AUTOTUNE_FORCE.  The characters end up holding
 * the solution of the last timed run.  best_ms is the winner's scaled
 * time; best and best_ms may be NULL. */
int mfs_autotune(mfs_context* ctx, int32_t count, mfs_character* const* chars,
                 const double* const* handle_R, const double* const* handle_t,
                 const mfs_solve_opts* opts, int32_t newton_iterations, const char* cache_path,
                 int32_t flags, mfs_tuning* best, double* best_ms);

/* ---- serving ------------------------------------------------------------ */

/* A request loop with continuous batching over one context.  A worker
 * thread owns the context's stream while the server exists: between
 * server_create and server_destroy the context and its characters are used
 * only through mfs_server_* calls (which may come from any host thread).
 * With lanes > 1 the server runs that many such loops at once, each with
 * its own worker thread, batch and stream (lane 0 on the caller's context,
 * the others on contexts the server creates on the same device with the
 * caller's PCG tuning, destroyed with the server); a request goes to the
 * first lane i whose lane_max_tets[i] is at least its character's tet count,
 * else to the last lane, so small characters are not held back by the long
 * PCG solves of large ones in a shared batch.  slots, queue_capacity and
 * workspace_budget_bytes hold per lane.
 * Each request is one frame solve (as mfs_solve_frame, with the server's
 * solve options).  Between Newton steps the worker admits queued requests
 * in submission order into free slots of the running batch; a request
 * waits while its character has a frame in flight (frames of a character
 * run in order, so MFS_WARM_PREVIOUS starts from the previous frame's
 * result) and, when its character released its workspace, until that
 * workspace fits in the server's device arena.  A request's result and
 * statistics do not depend on the other requests in the batch. */
typedef struct mfs_server mfs_server;

typedef struct mfs_server_opts {
  int32_t slots;                    /* frame solves in flight at once, 1..1024 */
  int32_t queue_capacity;           /* queued requests beyond which submit is MFS_E_BUSY */
  uint64_t workspace_budget_bytes;  /* device arena lent to requests whose character has no
                                       workspace of its own; 0 = no arena */
  mfs_solve_opts solve;             /* options of every solve; output_memory must be host */
  int32_t lanes;                    /* concurrent batches, 1..4 */
  int32_t reserved;                 /* 0 */
  int64_t lane_max_tets[3];         /* size-class bounds of lanes 0..lanes-2, increasing */
} mfs_server_opts;

typedef struct mfs_request_times {  /* seconds since the server was created (steady clock) */
  double submit_s;                  /* mfs_server_submit returned */
  double admit_s;                   /* the request joined the batch */
  double done_s;                    /* its result was copied out */
} mfs_request_times;

typedef struct mfs_server_info {
  int64_t submitted, completed;     /* requests so far */
  int64_t steps;                    /* batched Newton steps run */
  int32_t queued, running;          /* requests waiting / in the batch now */
  uint64_t arena_bytes;             /* arena capacity */
  uint64_t arena_in_use, arena_peak;
  double slot_steps;                /* sum over steps of requests in the batch
                                       (slot_steps / steps = mean batch width) */
} mfs_server_info;

/* slots 16, queue 4096, no arena, mfs_default_opts, one lane. */
void mfs_default_server_opts(mfs_server_opts* opts);
/* opts may be NULL (defaults).  Errors: MFS_E_INVALID, MFS_E_UNSUPPORTED,
 * MFS_E_OOM (arena), MFS_E_HIP. */
int mfs_server_create(mfs_context* ctx, const mfs_server_opts* opts, mfs_server** out);
/* Stops the worker after its current step; requests not yet taken are
 * dropped. */
int mfs_server_destroy(mfs_server* srv);
/* Queue one frame solve; the pose (n_handles x 9 and x 3, host) is copied
 * and validated as in mfs_solve_frame.  Returns at once with a ticket.
 * MFS_E_BUSY: queue full, or the request's workspace exceeds the arena. */
int mfs_server_submit(mfs_server* srv, mfs_character* ch, const double* handle_R,
                      const double* handle_t, uint64_t* ticket);
/* *done = 0 while the request is queued or running.  Once done, writes
 * x_out (n x 3 host, caller order), stats and times (each may be NULL),
 * forgets the ticket and returns the solve's status. */
int mfs_server_poll(mfs_server* srv, uint64_t ticket, double* x_out, mfs_solve_stats* stats,
                    mfs_request_times* times, int32_t* done);
/* As poll, blocking until the request is done. */
int mfs_server_wait(mfs_server* srv, uint64_t ticket, double* x_out, mfs_solve_stats* stats,
                    mfs_request_times* times);
/* Counters of the server; returns the worker's error if it stopped on one. */
int mfs_server_get_info(mfs_server* srv, mfs_server_info* info);
/* Sets the PCG schedule (as mfs_context_set_tuning) of one lane, 0..lanes-1;
 * a lane starts with the caller's context's schedule.  The lane's worker
 * applies it before its next Newton step, so frames in flight may run some
 * steps under each schedule.  Lets each size class run the schedule that
 * mfs_autotune chose for a batch of its characters.  Errors: MFS_E_INVALID
 * (lane out of range, a field out of range). */
int mfs_server_set_lane_tuning(mfs_server* srv, int32_t lane, const mfs_tuning* tuning);

/* ---- introspection and profiling ------------------------------------- */

typedef struct mfs_character_info {
  int64_t n_vertices, n_tets, n_blocks;  /* n, m, nonzero 3x3 blocks of K (both triangles) */
  int64_t n_pins;
  int32_t n_handles, reserved;
  double bbox_diag;                      /* rest bounding-box diagonal */
  double mean_edge;                      /* mean rest edge length */
} mfs_character_info;

/* Sizes of a created character. */
int mfs_character_get_info(const mfs_character* ch, mfs_character_info* info);

enum mfs_kernel_family {   /* kernel groups timed by the context profiler */
  MFS_K_WARM_START = 0,    /* polar-decomposition warm start */
  MFS_K_ELEMENT = 1,       /* per-element stretch, stress, Hessian state */
  MFS_K_ASSEMBLE = 2,      /* Schur-complement assembly (3x3 blocks, RHS, block Jacobi) */
  MFS_K_SPMV = 3,          /* PCG: search direction + block sparse matrix-vector product */
  MFS_K_CG_UPDATE = 4,     /* PCG: iterate / residual / preconditioner update */
  MFS_K_LINESEARCH = 5,    /* energy / feasibility evaluations */
  MFS_K_UPDATE = 6,        /* position and stretch updates */
  MFS_K_OTHER = 7,         /* PCG init/finish, reductions, permutations */
  MFS_K_FAMILIES = 8
};

typedef struct mfs_profile {
  double gpu_ms[MFS_K_FAMILIES];     /* summed HIP-event time of the timed launches */
  int64_t timed[MFS_K_FAMILIES];     /* launches that were timed */
  int64_t launches[MFS_K_FAMILIES];  /* all launches of the family */
  double bytes[MFS_K_FAMILIES];      /* algorithmic HBM bytes of the timed launches, counted
                                        for the systems a launch iterates (a system whose PCG
                                        stopped earlier in the run costs nothing).  SpMV family,
                                        per system with n block rows and nnzb blocks and w the
                                        solve's word size: the least a block-sparse product
                                        moves, nnzb (9 w + 4) + 4 (n + 1) + 6 w n (blocks,
                                        column indices, row pointers, one input and one output
                                        vector), plus 42 w n in the pipelined form, which fuses
                                        the PCG vector work and the block-Jacobi
                                        preconditioner (twelve passes over 3n values and six
                                        preconditioner values per row); 0 for families without
                                        a byte model */
} mfs_profile;

/* Time kernel launches of this context with HIP events on its stream:
 * every `stride`-th launch group of each family carries an event pair in
 * its kernel dispatches (start of the first kernel, end of the last), so a
 * timed interval is kernel execution only.  Timed runs launch kernels
 * directly instead of replaying graphs.  Stride 0 switches timing off and
 * clears the counters. */
int mfs_profile_enable(mfs_context* ctx, int32_t stride);

/* Synchronise the context's stream, fold the pending event pairs and copy
 * the counters; reset != 0 clears them afterwards. */
int mfs_profile_read(mfs_context* ctx, mfs_profile* out, int32_t reset);

/* ---- evaluation entry points (parity checks) --------------------------- */

/* At positions x (n x 3, caller order, host or device per memory_space) and
 * the given pose, with s = J x (the condensed stretch, sym(R_k^T F_k)):
 *   energy_out (1 double, host): E(x) = sum_k W_k Psi(S_k) + k_s/2 sum_p
 *       ||x_p - (R_h X_p + t_h)||^2 - f_ext . x (+inf if a neo-Hookean S_k
 *       is not positive definite);
 *   grad_out (n x 3, same memory space as x, or NULL): grad E(x);
 *   stretch_out (m x 6, same space, or NULL): s_k = (S00,S11,S22,S12,S02,S01)
 *       in the caller's tet order;
 * and, if v and Kv_out are non-NULL, Kv_out = K v with K the assembled
 * condensed matrix (Hessian of E, neo-Hookean clamp applied) in FP64. */
int mfs_evaluate(mfs_character* ch, const double* handle_R, const double* handle_t,
                 const double* x, const double* v, int32_t memory_space,
                 double* energy_out, double* grad_out, double* stretch_out, double* Kv_out);

/* Stress recovery (back-substitution of the stretch equations of Section 3):
 * at positions x (n x 3, caller order) and the given pose, per tet k in the
 * caller's tet order,
 *   stress_out (m x 6, or NULL): P_k = dPsi/dS at S_k = sym(R_k^T F_k(x)),
 *       stored (S00, S11, S22, S12, S02, S01);
 *   multiplier_out (m x 9 row-major, or NULL): lambda_k = W_k R_k P_k, the
 *       volume-weighted world-frame multiplier of the constraint F_k = R_k S_k
 *       (the element's force on its vertex a is lambda_k n_a, n_a the rest
 *       shape-function gradient).
 * Buffers host or device per memory_space.  A neo-Hookean tet whose S_k is not
 * positive definite gets NaN.  Uses the character's state buffers (its stored
 * solution is replaced by x, as in mfs_evaluate). */
int mfs_stress(mfs_character* ch, const double* handle_R, const double* handle_t, const double* x,
               int32_t memory_space, double* stress_out, double* multiplier_out);

/* mfs_evaluate without allocating: for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and memory spaces as
 * mfs_evaluate; it calls no hipMalloc, hipFree or other allocating routine.
 * Every buffer the evaluation needs beyond the caller's inputs and outputs
 * (the descriptor, the tile list, host staging, and the element records,
 * matrix values, right-hand side and partial sums of the evaluation) is
 * carved from one fixed array of 32 MiB in device memory that each GPU holds
 * from the first context created on it until the process ends; the
 * character's own workspace is neither used nor allocated.  A character
 * whose evaluation needs more than that (about 30k tets) is MFS_E_INVALID,
 * checked before any GPU work.  Calls on one GPU share the array: calls that
 * overlap on one GPU (from two streams or threads) race on it and must be
 * serialised by the caller.  The caller's arrays are read during the call
 * only, and the call synchronises the context's stream before returning. */
int mfs_evaluate_noalloc(mfs_character* ch, const double* handle_R, const double* handle_t,
                         const double* x, const double* v, int32_t memory_space,
                         double* energy_out, double* grad_out, double* stretch_out,
                         double* Kv_out);

/* Polar decomposition F = U P (U proper rotation, P symmetric) of `count`
 * 3x3 matrices by Higham's scaled Newton iteration, as the solver's warm
 * start uses it.  F, U: count x 9; P: count x 6 (S00,S11,S22,S12,S02,S01);
 * sigma_min: count (smallest eigenvalue of P); precision MFS_FP32_REFINED
 * runs FP32 and reroutes matrices with sigma_min < 1e-3 to FP64; routed:
 * count bytes (1 = ran in FP64), or NULL.  Matrices with det F <= 0 get
 * U = I, P = I, sigma_min = 0.  All buffers host or device per
 * memory_space. */
int mfs_polar(mfs_context* ctx, const double* F, int64_t count, int32_t precision,
              double* U, double* P, double* sigma_min, uint8_t* routed, int32_t memory_space);

#ifdef __cplusplus
}
#endif

#endif /* MFS_H */

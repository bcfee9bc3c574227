/*
 * dpml.h -- C ABI of the MI355X (gfx950) library for explicit time stepping
 * of the discrete scalar wave equation with the reflectionless discrete
 * perfectly matched layer of A. Chern, "A Reflectionless Discrete Perfectly
 * Matched Layer" (J. Comput. Phys.; arXiv 1804.01390).
 *
 * The scheme (per axis a, grid spacing h, shifts tau_a):
 *   Eq. (DiscretePML a):
 *     U_tt = c^2 sum_a (tau_a^-1 U - 2U + tau_a U)/h^2
 *            + sum_a (1/h)( sigma_a tau_a Psi_a - (tau_a^-1 sigma_a)(tau_a^-1 Phi_a) )
 *   Eq. (DiscretePML b):
 *     Phi_a,t = -1/2((tau_a^-1 sigma_a)(tau_a^-1 Phi_a) + sigma_a Phi_a) - (tau_a U - tau_a^-1 U)/(2h)
 *   Eq. (DiscretePML c):
 *     Psi_a,t = -1/2((tau_a^-1 sigma_a) Psi_a + sigma_a tau_a Psi_a) - (tau_a U - tau_a^-1 U)/(2h)
 * discretised in time by leapfrog for U and a forward step for Phi/Psi, every
 * right-hand side of a step taken from time level n:
 *   U^{n+1}   = 2U^n - U^{n-1} + dt^2 A(U^n, Phi^n, Psi^n)
 *   Phi^{n+1} = Phi^n + dt B(U^n, Phi^n),   Psi^{n+1} = Psi^n + dt C(U^n, Psi^n).
 * With this placement every discrete plane wave continues into the layer
 * exactly (Thm. 1 with omega' = i(z-1)/dt, z the one-step factor), so the
 * layer reflects nothing, for any damping profile.
 *
 * GRID AND LAYOUT.  Axis 0 (x) is fastest.  Axis a has n[a] interior cells
 * and lo[a] / hi[a] layer cells below / above them: N[a] = lo + n + hi cells,
 * interior [lo, lo+n).  The grid is periodic, so the two layer sides form one
 * band [lo+n, N) U [0, lo) traversed in +a direction (the "physical domain
 * surrounded by the layer" of the paper's runs, Sec. 1.1.3).  Fields U are
 * dense arrays of prod N[a] cells, cell (x,y,z) at x + N0*(y + N1*z).
 * sigma_a(i) belongs to the edge [i, i+1] and must vanish for i in [lo, lo+n).
 *
 * AUXILIARY LAYOUT (what dpml_field returns).  Phi_a and Psi_a are stored
 * only on the band (Sec. 1.1.2: Phi_a lives on {i_a >= 0}, Psi_a on
 * {i_a >= 1} in the paper's coordinates).  The band coordinate of index i is
 * j = (i - lo - n) mod N, j in [0, M], M = lo + hi (j = M is interior cell
 * lo).  The compact array for axis a has the same shape as U with extent
 * N[a] replaced by M+1 (x fastest); Phi_a is meaningful at j in [0, M-1],
 * Psi_a at j in [1, M]; the remaining slot of each stays 0.
 *
 * PRECISION.  dtype DPML_F32 or DPML_F64 for every device field; host tables
 * (sigma, c^2) are always FP64 and converted on upload.
 *
 * MEMORY.  The caller owns all large device memory: dpml_create borrows a
 * workspace of dpml_workspace_bytes() bytes (256-byte aligned) that must stay
 * alive until dpml_destroy.  The library itself allocates only the small
 * source/receiver index tables registered by dpml_inject / dpml_record.
 *
 * STREAMS.  All device work is enqueued on the HIP stream given to
 * dpml_create (NULL = the null stream), in call order.  Calls that return
 * device results do not synchronise unless stated.  A handle must be used by
 * one host thread at a time.
 *
 * ERRORS.  Every int-returning call returns DPML_OK (0) or a negative code;
 * no exception crosses the ABI.  dpml_last_error() gives a message.
 */
#ifndef DPML_H
#define DPML_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DPML_OK 0
#define DPML_EINVAL (-1)     /* invalid argument or unsupported configuration */
#define DPML_ENOMEM (-2)     /* workspace too small or allocation failed       */
#define DPML_EHIP (-3)       /* a HIP runtime call failed                      */
#define DPML_ESTATE (-4)     /* call not valid in the handle's current state   */
#define DPML_ENONFINITE (-5) /* a NaN or Inf appeared in the wave field        */

#define DPML_F32 0
#define DPML_F64 1

/* Field selectors for dpml_field. */
#define DPML_FIELD_U 0        /* U^n                                   */
#define DPML_FIELD_UPREV 1    /* U^{n-1}                               */
#define DPML_FIELD_PHI(a) (2 + 2 * (a))  /* Phi_a^n, compact band array */
#define DPML_FIELD_PSI(a) (3 + 2 * (a))  /* Psi_a^n, compact band array */

/* Kernel variants (dpml_set_variant); all compute identical results. */
#define DPML_VARIANT_AUTO 0   /* library default (CELL)                               */
#define DPML_VARIANT_CELL 1   /* one thread per cell; tile_rows = block rows TH in
                                 {1, 2, 4, 8} (block of 256/TH x TH cells)            */
#define DPML_VARIANT_MARCH 2  /* tiles marching along the slowest axis.  2D:
                                 tile_rows = rows per tile, the loads of 4 rows
                                 issued together.  3D periodic grids: one launch
                                 per step over the layer-free core and the three
                                 layer boxes, each wave holding 64 columns x RY
                                 rows of two planes in registers and taking every
                                 neighbour -- of U and of the layer fields -- from
                                 lanes, register rows or the previous plane
                                 (tile_rows: planes per core chunk in bits 0-11
                                 (0 = 64), RY of the core in bits 12-15 (1, 2, 4
                                 or 8; 0 = 4), RY of the z- and x-band boxes in
                                 bits 16-17 (0: 1, 1: 2, 2: 4; the y band takes
                                 1), the core's waves first bit 18, the core and
                                 the layer boxes as two launches on two streams
                                 bit 19, planes per layer chunk in bits 20-27
                                 (0 = 16); values below 2^30).  3D with walls:
                                 as MARCH1 with RY 4                              */
#define DPML_VARIANT_MARCH1 3 /* as MARCH; 2D: one row at a time; 3D: one z-march
                                 launch over the layer-free core (waves of 64
                                 columns x 2 rows, tile_rows planes per tile) and
                                 one thread per cell over the layer slabs         */
#define DPML_VARIANT_TWOSTEP 4 /* 2D runs without a recorded plane (with
                                  reflecting walls when every walled axis has a
                                  layer with a cell above the interior; with
                                  point sources or receivers single steps:
                                  FOURSTEP and DEEP take them inside their
                                  passes):
                                  two steps per pass over the layer-free core
                                  (temporal blocking: each wave marches down a
                                  strip keeping U^n and U^{n+1} rows in registers,
                                  2 words per cell per step; tile_rows: rows per
                                  wave in bits 0-11 (0 = 8), rows whose loads are
                                  issued together in bits 12-15 (1, 2 or 4; 0 = 2),
                                  rows per marching span of the frame's steps in
                                  bits 16-19 (0 = the frame one thread per
                                  cell)), the frame holding the layer in single
                                  steps.
                                  3D runs with a constant c^2, one batch member
                                  (walls as in 2D), x-y planes below 4 GiB and at
                                  most 32 sources, all at least 3 cells inside the
                                  layer-free region: the same
                                  with each wave marching in z over 64 columns x
                                  RY rows (tile_rows: planes per chunk in bits
                                  0-11 (0 = 32), RY in bits 12-17 (4, 8 or 16;
                                  0 = 8); the frame's steps by the box kernels,
                                  or with bit 19 on periodic axes by the
                                  register-neighbour march of MARCH (its planes
                                  per layer chunk in bits 20-27); the core's tiles in launch order bit
                                  28; bit 29: the frame's first step alone
                                  before the core, which then runs beside the
                                  frame's second step; bit 30 (periodic axes;
                                  with walls the frame's single steps by the box
                                  kernels and bits 18-29 ignored):
                                  the frame as two levels in one march per box
                                  beside the core -- the layer auxiliaries of
                                  the middle level stay in registers, the core
                                  writes U^{n+1} on all of its cells -- with RY
                                  of the boxes outside the core along one axis
                                  in bit 18 (0: 2, 1: 4; the others take 2),
                                  the boxes outside along two or three axes on
                                  the core's stream after it with bit 19,
                                  planes per chunk of those boxes in bit 20
                                  (0: 8, 1: 4) and of the x and y boxes in bits
                                  21-25 (in eights; 0 = 32), chunks of the z
                                  box in bits 26-27 (1, 2, 4 or 8) and with bit
                                  29 the layer arrays loaded at their own plane
                                  instead of a plane ahead);
                                  sources are added inside the pass, receivers
                                  and planes recorded after it.
                                  Otherwise single steps as CELL (2D) or MARCH
                                  (3D)                                                */
#define DPML_VARIANT_THREESTEP 5 /* 2D: as TWOSTEP with three steps per pass over a
                                  core one cell smaller (4 words per cell per three
                                  steps: U^{n+1} stays in registers and U^{n+2} is
                                  stored off the core's boundary ring, where the
                                  frame's steps write it; tile_rows as for
                                  TWOSTEP); a remaining pair takes the two-step
                                  pass.  3D: as TWOSTEP                            */
#define DPML_VARIANT_FOURSTEP 6  /* 2D: as THREESTEP with four steps per pass over a
                                  core one cell smaller again (4 words per cell per
                                  four steps: U^{n+1} and U^{n+2} stay in
                                  registers, U^{n+3} is stored off the core's
                                  boundary ring); remaining steps take the three-
                                  or two-step pass.  3D: as TWOSTEP               */
#define DPML_VARIANT_DEEP 7      /* 2D: as FOURSTEP with D steps per pass, D in
                                  bits 20-23 of tile_rows (2 .. 8; 0 = 6): the
                                  core keeps U^{n+1} .. U^{n+D-2} in registers and
                                  stores U^{n+D-1} off its boundary ring and
                                  U^{n+D} on it (4 words per core cell per D
                                  steps) over a core [lo+D, lo+n+1-D) per axis;
                                  the frame takes D single steps beside it; the
                                  last steps of a run take a shorter pass.  Bit
                                  24: depths 4 .. 8 take every march index's
                                  loads from a ring issued four indices ahead.  The lower bits as for TWOSTEP,
                                  and frame form 15 in bits 16-19 (any multi-step
                                  variant) takes all the frame's steps of a pass
                                  in one launch over tiles held in LDS with a
                                  halo of D cells.  With point sources or
                                  receivers (2D): passes of 4 .. 8 levels when
                                  at most 32 sources are registered, each at
                                  least D-1 cells inside the core, no two
                                  receivers share a cell and the frame is not
                                  fused; the core adds the sources at every
                                  level it forms and records the receivers at
                                  least D-l cells inside it at level l, the
                                  frame's steps the rest; otherwise shallower
                                  passes or single steps.  3D: as TWOSTEP        */

typedef struct dpml_grid {
    int32_t ndim;    /* 2 or 3 */
    int32_t dtype;   /* DPML_F32 or DPML_F64 */
    int64_t n[3];    /* interior cells per axis (unused axes: 1) */
    int32_t lo[3];   /* layer cells below the interior (unused axes: 0) */
    int32_t hi[3];   /* layer cells above the interior (unused axes: 0) */
    int64_t batch;   /* independent problems of this grid stepped together
                        (shots sharing c^2 and sigma); <= 1 means one.  Every
                        device field is then [batch][member] with the member
                        layout below; cell indices passed to dpml_inject /
                        dpml_record address the whole batch
                        (member * prod N + cell). */
    int32_t walls[3];/* per axis: 0 = periodic wrap (the layer sides form one
                        band, the paper's runs); 1 = reflecting walls: U, Phi
                        and Psi vanish on ghost cells -1 and N, and the ghost
                        edge [-1, 0] is undamped (the truncation the paper
                        bounds with Eq. (IntroReflectedDecayBound)).  Walls
                        are supported by dpml_step only (not by the adjoint,
                        RK4 or multi-problem paths: DPML_EINVAL there). */
    int32_t reserved;
} dpml_grid_t;

typedef struct dpml dpml_t;

/* Bytes of device workspace dpml_create needs for grid g; c2_is_field != 0
 * when c^2 will be given per cell.  Returns 0 for an invalid grid. */
size_t dpml_workspace_bytes(const dpml_grid_t *g, int32_t c2_is_field);

/* Create a stepper (Eq. (DiscretePML) with the time placement above).
 *   h, dt    grid spacing and time step (> 0).
 *   c2       host FP64: c2_len == 1 (constant) or prod N[a] values (per cell).
 *            c^2 multiplies the Laplacian only and must be 1 on every layer
 *            cell and within one cell of the layer (unit speed where damping
 *            acts, as in the paper).
 *   sigma    host FP64 arrays sigma[a] of N[a] values for a < ndim (NULL for
 *            an axis means no damping on it).  sigma >= 0, finite, zero on the
 *            interior indices [lo, lo+n).  Any profile is reflectionless
 *            (Sec. 1.1.3, the remark after Thm. 1).
 *   workspace, ws_bytes  caller-owned device memory (borrowed).
 *   stream   hipStream_t for all work of this handle.
 * Host arrays are copied; the caller may free them on return.
 * Errors: DPML_EINVAL for ndim/dtype/extents out of range, non-positive h/dt,
 * c_max dt/h sqrt(ndim) > 1 (leapfrog stability), dt max(sigma) > 4
 * (forward-step stability of the auxiliaries), bad sigma or c^2 values;
 * DPML_ENOMEM if ws_bytes is too small or workspace is not 256-byte aligned;
 * DPML_EHIP on a runtime failure.  On error *out is set to NULL. */
int dpml_create(const dpml_grid_t *g, double h, double dt,
                const double *c2, int64_t c2_len,
                const double *const sigma[3],
                void *workspace, size_t ws_bytes, void *stream,
                dpml_t **out);

/* Set the initial state (time index 0): U^0 = U0, Phi = Psi = 0 and
 * U^{-1} = U^0 - dt V^0 + dt^2/2 A(U^0), the start that is exact for
 * Fourier modes at rest.  U0, V0: device arrays of the grid's dtype and
 * prod N[a] cells (V0 == NULL: zero initial velocity, as in the paper's
 * runs).  Read on the stream; they may be released once the stream passes
 * this point. */
int dpml_set_state(dpml_t *h, const void *U0, const void *V0);

/* Register point sources (not part of the paper): after step n the value
 * dt^2 w_s[n] / h^ndim is added to U^{n+1} at cell cells[s].
 *   cells     host int64 flat cell indices (copied), 0 <= cell < prod N.
 *   wavelets  device [ns][nt] array in dtype (borrowed until replaced).
 * ns == 0 removes all sources.  Replaces earlier registrations. */
int dpml_inject(dpml_t *h, int64_t ns, const int64_t *cells,
                const void *wavelets, int64_t nt);

/* Register point receivers: after step n (and its sources), traces[r][n] =
 * U^{n+1}[cells[r]] for n < nt.  cells: host int64 (copied); traces: device
 * [nr][nt] in dtype (borrowed).  nr == 0 removes receivers. */
int dpml_record(dpml_t *h, int64_t nr, const int64_t *cells, void *traces,
                int64_t nt);

/* Register a recorded plane: after step n, planes[n] = U^{n+1} on the plane
 * i_axis = index (x-fastest order of the remaining axes).  planes: device
 * [nt][plane cells] in dtype (borrowed).  axis < 0 removes the recorder. */
int dpml_record_plane(dpml_t *h, int32_t axis, int64_t index, void *planes,
                      int64_t nt);

/* Choose the kernel variant (DPML_VARIANT_*) and its launch shape
 * tile_rows (meaning per variant above; 0 = default).  All variants
 * evaluate the scheme in the same operation order, so results do not
 * depend on the choice.  DPML_EINVAL for an unknown variant or tile_rows
 * outside [0, 2^20) ([0, 2^25) for DEEP, whose depth may not be 1; [0, 2^30)
 * for MARCH and the multi-step variants on a 3D grid). */
int dpml_set_variant(dpml_t *h, int32_t variant, int32_t tile_rows);

/* Enqueue nsteps fused steps (U, Phi, Psi, sources, receivers).  Returns
 * before the work completes.  DPML_ESTATE before dpml_set_state;
 * DPML_EINVAL if nsteps < 0. */
int dpml_step(dpml_t *h, int64_t nsteps);

/* As dpml_step for a run without sources, receivers or planes (DPML_EINVAL
 * otherwise), but the nsteps launches are captured once into a HIP graph
 * (cached for the same nsteps, buffer parity and kernel variant) and
 * replayed with a single launch: for small grids whose steps are shorter
 * than a kernel launch. */
int dpml_step_graph(dpml_t *h, int64_t nsteps);

/* As dpml_step, but every `every` steps (and at the end) synchronises and
 * scans U^n for NaN/Inf; returns DPML_ENONFINITE at the first hit (the state
 * is left at that step). */
int dpml_step_checked(dpml_t *h, int64_t nsteps, int64_t every);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * dpml_step_checked, but the call allocates nothing -- no hipMalloc, no
 * stream, event or table created on first use.  Steps are taken one at a
 * time by the one-thread-per-cell kernel (whatever dpml_set_variant chose;
 * results are identical), sources and receivers from the tables registered
 * beforehand, and the non-finite scan keeps its flags (one int32 per scan
 * block, 1024 of them, 4 KiB) in a static device array of the library that
 * each GPU holds until the process ends.  Calls that overlap on one GPU (from
 * several threads or handles) share that array and race.  The scan strides
 * over the grid, so any grid dpml_create accepts is handled (up to 2^40
 * cells; larger gives DPML_EINVAL).  Return codes as dpml_step_checked. */
int dpml_step_checked_noalloc(dpml_t *h, int64_t nsteps, int64_t every);

/* Borrowed device pointer to a field of the current time level (see the
 * DPML_FIELD_* selectors and the auxiliary layout above) and its extents in
 * x, y, z order (unused axes 1).  Valid until the next dpml_step. */
int dpml_field(dpml_t *h, int32_t which, void **ptr, int64_t shape[3]);

/* Time index n of the current level U^n. */
int64_t dpml_time_index(const dpml_t *h);

/* Checkpoint / resume: dpml_state_bytes() bytes of device memory hold U^n,
 * U^{n-1} and every Phi_a, Psi_a.  dpml_get_state copies the state out,
 * dpml_put_state restores it with time index n (stream-ordered).  A resumed
 * run is bit-identical to an uninterrupted one. */
size_t dpml_state_bytes(const dpml_t *h);
int dpml_get_state(dpml_t *h, void *blob);
int dpml_put_state(dpml_t *h, const void *blob, int64_t n);

/* ---- Discrete adjoint (reverse mode of the scheme above) ----------------
 * For the receiver misfit J = 1/2 sum_{r,n} (traces[r][n] - obs[r][n])^2 the
 * adjoint of one step is the transposed step, run backwards in time:
 *   a^n   = 2a^{n+1} - a^{n+2} + dt^2 L(c^2 a^{n+1}) + dt sum_a G_a(p_a + q_a)
 *   p_a^n = p_a - dt/2 sigma(i)(p_a(i) + p_a(i+e)) - dt^2/h sigma(i) a^{n+1}(i+e)
 *   q_a^n = q_a - dt/2 sigma(i-1)(q_a(i) + q_a(i-e)) + dt^2/h sigma(i-1) a^{n+1}(i-e)
 * (a, p, q adjoint to U, Phi, Psi; G_a the central difference, L the
 * Laplacian), giving dJ/dc^2 = sum_n dt^2 a^{n+1} L U^n (+ the start term)
 * and dJ/dw_s[n] = dt^2/h^d a^{n+1}(s).  Forward levels are recomputed from
 * checkpoints taken every ckpt_every steps (sqrt(T) checkpointing). */

/* Bytes of caller-owned device memory the checkpointed forward + adjoint of
 * nsteps steps needs (checkpoints, two segments of recomputed levels -- the
 * next segment is recomputed on streams of the library's own while the
 * current one is swept -- and the adjoint state).  0 on invalid arguments.  The adjoint recomputes each
 * segment with the handle's variant (2D multi-step passes keep every level
 * they form, writing it straight into the segment's history), so results
 * do not depend on the variant. */
size_t dpml_adjoint_workspace_bytes(const dpml_t *h, int64_t nsteps, int64_t ckpt_every);

/* Run nsteps steps from time index 0 (after dpml_set_state) exactly as
 * dpml_step does (sources, receivers, plane), saving a checkpoint of the
 * state every ckpt_every steps into adj_ws (borrowed until the next call of
 * this function).  DPML_ESTATE if the handle is not at time index 0. */
int dpml_forward_checkpointed(dpml_t *h, int64_t nsteps, int64_t ckpt_every,
                              void *adj_ws, size_t bytes);

/* Gradients of J after dpml_forward_checkpointed:
 *   resid    device [nr][nt] in dtype: traces - obs for the registered
 *            receivers (same layout as the trace buffer);
 *   grad_c2  device FP64, prod N values, ACCUMULATED (+=) over all batch
 *            members and steps (FP64 accumulation, deterministic);
 *   grad_w   device [ns][nt] in dtype for the registered sources (written
 *            for n < nsteps), or NULL.
 * Afterwards the handle's fields hold an intermediate level: call
 * dpml_set_state or dpml_put_state before stepping again.  May be called
 * again (e.g. with another residual) while the checkpoints are intact. */
int dpml_adjoint(dpml_t *h, const void *resid, double *grad_c2, void *grad_w);

/* Wait for the handle's stream and report any deferred HIP error. */
int dpml_sync(dpml_t *h);

/* ---- The paper's own integrator: RK4 ---------------------------------------
 * Classic fourth-order Runge-Kutta on the first-order system U_t = V,
 * V_t = A(U, Phi, Psi), Phi_a,t = B_a, Psi_a,t = C_a with the right-hand
 * sides of Eq. (DiscretePML a, b, c) (the time stepping of the paper's runs,
 * Sec. 1.1.3).  Exactly reflectionless as well: the continued plane waves of
 * Thm. 1 are eigenvectors of the semi-discrete system, hence of any
 * polynomial one-step map.  Four fused stage sweeps per step.  Uses the
 * handle's grid, damping tables and c^2 (batch must be 1); its state lives in
 * a separate caller-owned workspace; no sources or receivers. */

/* Bytes of that workspace (four copies of U, V, Phi_a, Psi_a); 0 if the
 * handle has batch > 1. */
size_t dpml_rk4_workspace_bytes(const dpml_t *h);

/* Bind the workspace (borrowed, 256-byte aligned) and set U = U0,
 * V = V0 (NULL: zero), Phi = Psi = 0; RK4 time index 0. */
int dpml_rk4_set_state(dpml_t *h, void *rk_ws, size_t bytes, const void *U0, const void *V0);

/* Enqueue nsteps RK4 steps (asynchronous). */
int dpml_rk4_step(dpml_t *h, int64_t nsteps);

/* Borrowed pointer/extents of the RK4 state: which = DPML_FIELD_U (U),
 * 1 (V = U_t), DPML_FIELD_PHI(a), DPML_FIELD_PSI(a) (compact, as above). */
int dpml_rk4_field(dpml_t *h, int32_t which, void **ptr, int64_t shape[3]);

/* RK4 step count since dpml_rk4_set_state, or -1. */
int64_t dpml_rk4_time_index(const dpml_t *h);

/* ---- Many independent 2D problems of different sizes --------------------
 * Each problem is its own grid (Eq. (DiscretePML) with unit wave speed, the
 * time placement above and its own h, dt, sigma); one kernel launch per step
 * advances every problem, walking a flat work list of row tiles over all of
 * them, and a whole run of steps can be captured into one HIP graph and
 * replayed by a single launch.  No sources/receivers on this path. */
typedef struct dpml_multi dpml_multi_t;

/* Workspace bytes for `count` problems (grids[p].ndim must be 2, one dtype
 * for all, batch <= 1).  0 on invalid grids. */
size_t dpml_multi_workspace_bytes(int64_t count, const dpml_grid_t *grids);

/* Create.  h[p], dt[p] per problem (dt/h sqrt(2) <= 1, dt max sigma <= 4);
 * sigmas[3p + a] the host FP64 damping array of axis a (a = 0, 1; entry
 * 3p + 2 unused), same rules as dpml_create.  Host arrays are copied;
 * workspace is borrowed (256-byte aligned); all work goes on `stream`.
 * Errors as dpml_create (message from dpml_multi_last_error(NULL)). */
int dpml_multi_create(int64_t count, const dpml_grid_t *grids, const double *h,
                      const double *dt, const double *const *sigmas,
                      void *workspace, size_t ws_bytes, void *stream,
                      dpml_multi_t **out);

/* Start every problem at rest: U0[p] is a device array of problem p's
 * dtype and cells (read on the stream). */
int dpml_multi_set_state(dpml_multi_t *h, const void *const *U0);

/* Advance all problems nsteps steps.  use_graph != 0 captures the nsteps
 * launches into one HIP graph (cached for the same nsteps and buffer parity)
 * and replays it with one launch. */
int dpml_multi_step(dpml_multi_t *h, int64_t nsteps, int32_t use_graph);

/* Borrowed pointer and extents of a field of problem `prob` (selectors and
 * layouts as dpml_field). */
int dpml_multi_field(dpml_multi_t *h, int64_t prob, int32_t which, void **ptr,
                     int64_t shape[3]);

/* Tiles in the work list of one step (for reporting). */
int64_t dpml_multi_tiles(const dpml_multi_t *h);

/* Stepping scheme and launch shape of the many-problem path.
 *   DPML_VARIANT_MARCH (or AUTO; the default): single steps, each tile 256
 *     (FP32 with even widths: 512) columns x tile_rows rows of one problem
 *     marched down with the loads of `group` rows issued together;
 *     tile_rows in [4, 4096] (0: 32), group 1, 2 or 4 (0: 4).
 *   DPML_VARIANT_TWOSTEP: two steps per pass (if every problem has a core
 *     free of damping terms two cells deep; otherwise single steps): the
 *     cores of all problems in one launch (each wave marches a strip of
 *     tile_rows rows keeping U^n and U^{n+1} rows in registers, `group` rows
 *     of loads at a time; tile_rows in [1, 4096] (0: 8), group 0: 2), the
 *     frames of all problems as two single steps on a second stream
 *     meanwhile; an odd last step is a single step.
 *   DPML_VARIANT_THREESTEP: as TWOSTEP with three steps per pass over cores
 *     one cell smaller (U^{n+1} kept in registers), three frame steps, and
 *     a two-step pass for a remaining pair.
 *   DPML_VARIANT_FOURSTEP: four steps per pass over cores one cell smaller
 *     again (U^{n+1} and U^{n+2} kept in registers), four frame steps, and
 *     a three- or two-step pass for the remaining steps.
 *   DPML_VARIANT_DEEP: passes of D levels, D in bits 20-23 of tile_rows
 *     (2 .. 8; 0 = 6), tile_rows' low 20 bits as for TWOSTEP.
 * Results do not depend on the choice.  Drops a captured graph.
 * DPML_EINVAL for another variant or a shape out of range. */
int dpml_multi_set_variant(dpml_multi_t *h, int32_t variant, int32_t tile_rows, int32_t group);

int dpml_multi_sync(dpml_multi_t *h);
void dpml_multi_destroy(dpml_multi_t *h);
const char *dpml_multi_last_error(const dpml_multi_t *h);

/* ---- launch timing (measurement) ------------------------------------------
 * With timing on, the library brackets every launch of a step kernel with a
 * pair of HIP events on the handle's stream and records, per kernel class,
 * the launch count, the summed launch durations and the summed algorithmic
 * bytes of those launches (the byte model of the roofline: 3 words per cell
 * per step, 4 words per layer axis-cell per step, 1 word per cell per step
 * of a c^2 field; the core launch of a multi-step pass counts what the pass
 * must move whatever its depth -- 4 words per core cell (U^n, U^{n-1} read,
 * the pass's last two levels written) plus 1 word per cell of a c^2 field --
 * and a fused frame launch counts its cells once per level it advances).  Launches
 * inside a HIP-graph capture are not timed; at most 4096 launches are kept
 * between two reads.  Frame launches run on a second stream beside the core
 * launch, so their durations include time shared with it.  The events
 * slightly delay back-to-back launches, so throughput should be timed with
 * timing off. */
#define DPML_KERNEL_STEP 0   /* one step over all cells (any variant)                */
#define DPML_KERNEL_PAIR 1   /* the core kernel of a multi-step pass (any depth)     */
#define DPML_KERNEL_FRAME 2  /* the frame's steps of a multi-step pass (one launch
                                per step, or one fused launch per pass); the layer
                                slabs of a split 3D marching step                   */
#define DPML_KERNEL_CORE 3   /* the marching box of a split 3D marching step        */

typedef struct dpml_timing {
    int64_t launches[4];     /* indexed by DPML_KERNEL_*                               */
    double ms[4];            /* summed launch durations, milliseconds                  */
    double bytes[4];         /* summed algorithmic bytes                               */
} dpml_timing_t;

/* Turn launch timing on (enable != 0; clears earlier records) or off (keeps
 * them for dpml_get_timing).  DPML_EINVAL for a NULL handle. */
int dpml_set_timing(dpml_t *h, int32_t enable);

/* Wait for the recorded launches, write their per-class totals to *out and
 * clear the records.  Returns DPML_EHIP if an event query fails. */
int dpml_get_timing(dpml_t *h, dpml_timing_t *out);

/* ---- streaming bandwidth probe (measurement) -------------------------------
 * Not part of the paper: a plain streaming kernel over one device buffer,
 * timed with HIP events, that states the HBM bandwidth the stencil kernels
 * can reach and calibrates the hardware traffic counters against a kernel
 * of known size.
 *   kind    DPML_PROBE_READ (read `bytes` of src; one 16-byte XOR fold per
 *           block is written to dst, which must hold DPML_PROBE_MAX_BLOCKS
 *           x 16 bytes), DPML_PROBE_WRITE (write `bytes` of dst; src unused)
 *           or DPML_PROBE_COPY (dst = src, `bytes` each way), optionally or-ed
 *           with DPML_PROBE_NONTEMPORAL (non-temporal loads and stores).
 *   bytes   a positive multiple of 16; src and dst 16-byte aligned device
 *           pointers (borrowed for the call).
 *   blocks_per_cu  256-thread blocks per compute unit (1 .. 64); the grid
 *           never exceeds one block per 256 elements.
 *   reps    launches timed back to back on `stream` (hipStream_t).
 * Waits for the launches; *ms_per_rep = elapsed milliseconds / reps.
 * DPML_EINVAL for bad arguments, DPML_EHIP on a runtime failure. */
#define DPML_PROBE_READ 0
#define DPML_PROBE_WRITE 1
#define DPML_PROBE_COPY 2
#define DPML_PROBE_NONTEMPORAL 4
#define DPML_PROBE_MAX_BLOCKS 16384

int dpml_bandwidth_probe(int32_t kind, void *dst, const void *src, size_t bytes, int32_t blocks_per_cu,
                         int32_t reps, void *stream, double *ms_per_rep);

/* Release the handle (not the caller's workspace or buffers). */
void dpml_destroy(dpml_t *h);

/* Message for an error code, and the last detailed message of a handle
 * (or of the last failed dpml_create when h == NULL). */
const char *dpml_strerror(int code);
const char *dpml_last_error(const dpml_t *h);

#ifdef __cplusplus
}
#endif

#endif /* DPML_H */

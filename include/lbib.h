/*
 * lbib: lattice Boltzmann - Kinematic / Dynamic immersed boundary solver for
 * deformable capsules on one AMD MI355X (gfx950).
 *
 * Method: Coclite, Ranaldo, de Tullio, Decuzzi, Pascazio, "Kinematic and
 * Dynamic Forcing Strategies for Predicting the Transport of Inertial Capsules
 * via a combined Lattice Boltzmann - Immersed Boundary Method",
 * arXiv:1903.03356.  Section and equation numbers below refer to that paper.
 *
 * Conventions for every call
 *  - Plain C ABI.  Every call returns an lbib_status (0 = success, < 0 =
 *    error).  No C++ exception and no abort crosses the ABI.  On error,
 *    lbib_last_error() describes the cause.
 *  - Lattice units: dx = dt = 1, reference density 1, c_s^2 = 1/3,
 *    viscosity nu = (tau - 1/2)/3 (Sec. 2.1).
 *  - D2Q9 population order (Eq. 3): 0 rest; 1..4 = E, N, W, S; 5..8 = NE, NW,
 *    SW, SE.
 *  - Field arrays exchanged through get/set use the layout
 *    [component][y][x] (x fastest), FP64.  Capsule node arrays are
 *    [node][2] (x, y), FP64.
 *  - The library never allocates device memory.  The caller allocates the
 *    buffers listed by lbib_buffer_id, with the sizes given by
 *    lbib_required_bytes, and binds them at lbib_create.  They remain
 *    owned by the caller and must outlive the context.  Host arrays passed
 *    in are copied before the call returns.
 *  - Work is queued on the HIP stream bound at lbib_create.  Calls do not
 *    synchronise, except: get/set with a host pointer, lbib_check and
 *    lbib_get_timing.  Those wait for the stream.
 */
#ifndef LBIB_H
#define LBIB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbib_ctx lbib_ctx;

typedef enum {
    LBIB_OK = 0,
    LBIB_EINVAL = -1,    /* invalid argument (size, range, orientation, non-finite value) */
    LBIB_ECAPACITY = -2, /* capsule / node capacity exceeded, buffer too small */
    LBIB_EDEVICE = -3,   /* a HIP runtime call failed */
    LBIB_ESTATE = -4,    /* call not allowed in the current state */
    LBIB_ENUMERIC = -5   /* the device raised a status flag (see lbib_device_flags) */
} lbib_status;

/* Coupling scheme, fixed for the life of a context after the first step.
 * KINEMATIC: Sec. 2.4, steps i-viii, node update Eq. 25 (density ratio 1).
 * DYNAMIC:   Sec. 2.3.2, steps 1-8, Newton law Eqs. 21-22, Verlet Eq. 23,
 *            BDF2 node velocity Eq. 24. */
typedef enum { LBIB_KINEMATIC = 0, LBIB_DYNAMIC = 1 } lbib_mode;

/* Status bits raised by the device.  lbib_check returns LBIB_ENUMERIC if any
 * is set: */
enum lbib_device_flags {
    LBIB_FLAG_WALL = 1,       /* an MLS support touched a wall row (needs 1 <= y <= ny-2) or an
                                 open-channel inlet / outlet column */
    LBIB_FLAG_NONFINITE = 2,  /* a node position or staged density is NaN/Inf */
    LBIB_FLAG_PATCH = 4,      /* a capsule's fluid patch exceeded the on-chip capacity */
    LBIB_FLAG_OVERFLOW = 8,   /* a spread force left the fixed-point range (|f| >= 2^14) */
    LBIB_FLAG_MOVE = 16,      /* a node moved one lattice unit or more in one step */
    LBIB_FLAG_NEAR = 32,      /* overlapped schedule: an IB force outside the near regions */
    LBIB_FLAG_SYNC = 64,      /* overlapped schedule: a far-pass block stopped waiting for the IB
                                 launch of its step (about 0.05 s); that step is not valid */
    LBIB_FLAG_EDGE = 128,     /* an element longer than the limit of lbib_set_limits */
    LBIB_FLAG_AREA = 256      /* |A / A0 - 1| beyond the limit of lbib_set_limits */
};

typedef struct {
    int32_t nx, ny;            /* lattice nodes; walls are the rows y = 0 and y = ny-1 */
    int32_t real_bytes;        /* 4: FP32 populations and node offsets, 8: FP64 */
    int32_t max_capsules;      /* capacity of the capsule table (>= 1) */
    int32_t max_nodes_total;   /* capacity of the node arrays, all capsules (>= 3) */
    int32_t max_nodes_capsule; /* largest node count of any one capsule (3..2048) */
} lbib_grid;

typedef struct {
    int32_t periodic_x;     /* 1: x is periodic; 0: open channel (Sec. 3.2): Zou-He velocity inlet at
                               x = 0 with u_x = 4 inlet_umax y (H - y) / H^2, u_y = 0, and Zou-He
                               pressure outlet at x = nx-1 with rho = outlet_rho; needs stationary
                               walls (periodic_y = 0, wall speeds 0) and body_force_x = 0.  Corner
                               nodes: bounce-back of the non-equilibrium part, the two buried
                               populations share the mass deficit with the density of the inner
                               diagonal neighbour.  Capsule nodes must keep 3 <= x <= nx - 4 */
    int32_t periodic_y;     /* 1: fully periodic box; 0: Zou-He walls at y = 0, ny-1 (Sec. 2.1, ref. [36]) */
    double u_bottom, u_top; /* tangential wall speeds (lattice units) */
    double body_force_x;    /* uniform body force g added to the IB force everywhere (0 for none) */
    int32_t init_profile;   /* initial velocity: 0 rest, 1 linear between the wall speeds,
                               2 body-force Poiseuille g/(2 nu) y (H - y), H = ny - 1,
                               3 uniform (init_ux, init_uy), 4 the inlet parabola (open channel) */
    double init_ux, init_uy;
    double inlet_umax;      /* open channel: peak inlet speed */
    double outlet_rho;      /* open channel: outlet density, (0.5, 2) */
} lbib_walls;

/* Caller-owned device buffers, bound at lbib_create in this order. */
typedef enum {
    LBIB_BUF_POPS_A = 0, /* populations, ping */
    LBIB_BUF_POPS_B = 1, /* populations, pong */
    LBIB_BUF_FORCE = 2,  /* IB force field, two time levels, fixed point */
    LBIB_BUF_FLAGS = 3,  /* active-segment flags of the force field */
    LBIB_BUF_NODES = 4,  /* per-node capsule state */
    LBIB_BUF_CAPS = 5,   /* per-capsule records */
    LBIB_BUF_DIAG = 6,   /* per-capsule FP64 diagnostics and the device status word */
    LBIB_BUF_STAGE = 7,  /* staging for host transfers and layout conversion */
    LBIB_NUM_BUFFERS = 8
} lbib_buffer_id;

/* What lbib_get_state / lbib_set_state transfer. */
typedef enum {
    LBIB_F_POPS = 0,      /* f^n after streaming and walls, [9][ny][nx]                     (get, set) */
    LBIB_F_POPS_DEV = 1,  /* f^n - w_i (deviation from the rest weights), [9][ny][nx]        (get) */
    LBIB_F_MOMENTS = 2,   /* rho, ux, uy [3][ny][nx]; u = (sum f e + F^{n-1}/2)/rho (Eqs. 6-7) (get) */
    LBIB_F_FORCE = 3,     /* total force F^{n-1} = f_ib + g of the last collision [2][ny][nx] (get) */
    LBIB_C_NODES = 4,     /* x^n of one capsule [nv][2]                                       (get) */
    LBIB_C_PREV = 5,      /* x^{n-1} [nv][2]                                                   (get) */
    LBIB_C_VEL = 6,       /* u_v^n (Eq. 24; Dynamic) [nv][2]                                   (get) */
    LBIB_C_FORCE = 7,     /* last nodal force: total (Dynamic) or internal (Kinematic) [nv][2] (get) */
    LBIB_C_STATE = 8,     /* x^n, x^{n-1}, u_v^n stacked, [3][nv][2]                           (get, set) */
    LBIB_C_DIAG = 9,      /* 16 FP64 values, see lbib_diag_index                              (get) */
    LBIB_STATUS = 10,     /* int32 device status word (lbib_device_flags)                     (get) */
    LBIB_C_RIGID = 11     /* rigid particle: 10 FP64 values X, Y, theta, u_x, u_y, omega, F_x, F_y,
                             M (last load), rigid flag; host memory only                       (get) */
} lbib_state_id;

/* Layout of the LBIB_C_DIAG record (Sec. 3.1-3.2 diagnostics, all FP64). */
enum lbib_diag_index {
    LBIB_D_AREA = 0,      /* enclosed area A (Green's theorem) */
    LBIB_D_PERIMETER = 1, /* perimeter P */
    LBIB_D_CX = 2,        /* area centroid x */
    LBIB_D_CY = 3,        /* area centroid y */
    LBIB_D_TAYLOR = 4,    /* Taylor deformation (a - b)/(a + b), a, b from the area second moments */
    LBIB_D_SWELLING = 5,  /* swelling ratio A / (P^2 / 4 pi) */
    LBIB_D_DPERIM = 6,    /* perimeter variation (P - P0)/P0 */
    LBIB_D_DAREA = 7,     /* A / A0 - 1 */
    LBIB_D_JXX = 8,       /* central second moments of area */
    LBIB_D_JYY = 9,
    LBIB_D_JXY = 10,
    LBIB_D_A0 = 11,
    LBIB_D_P0 = 12
};

/* Size in bytes of buffer `buffer_id` for this grid, or 0 if the grid is
 * invalid.  Allocate each buffer with at least this many bytes, 256-byte aligned. */
size_t lbib_required_bytes(const lbib_grid* grid, int32_t buffer_id);

/* Creates a context on the current HIP device (Sec. 2.1 lattice, Sec. 2.2 forcing).
 * tau > 1/2 is the BGK relaxation time (Eq. 1).  device_buffers[LBIB_NUM_BUFFERS]
 * are caller-owned device pointers sized by lbib_required_bytes.  hip_stream is a
 * hipStream_t (NULL = the default stream).
 * The call zeroes the force and flag buffers and writes the initial
 * populations f^0 = f^eq(1, u_init) (Eq. 2), queued on the stream.
 * Errors: EINVAL (nx or ny < 8, tau <= 1/2, periodic_x not 0 or 1, an open channel
 * with moving or periodic walls or a body force, real_bytes not 4 or 8,
 * non-finite values, NULL buffers), ECAPACITY (capacities out of range, or a
 * max_nodes_capsule whose node arrays leave the IB kernel's on-chip memory too
 * little room for a fluid patch: on MI355X about 1100 nodes in FP32, 500 in FP64),
 * EDEVICE (HIP failure).  *out is set only on success. */
lbib_status lbib_create(const lbib_grid* grid, double tau, const lbib_walls* walls,
                        void* const* device_buffers, int32_t n_buffers, void* hip_stream,
                        lbib_ctx** out);

/* Adds one closed capsule membrane (Sec. 2.2, 2.2.1).  nodes_xy: host array
 * [n][2] FP64, counter-clockwise.  The given shape is the stress-free one,
 * from which it takes l0, theta0, A0 and P0.
 * ks: n_ks = 1 (uniform) or n (element l joins node l to l+1) stretching
 * constants (Eq. 10).  kb: bending constant (Eqs. 12-13).  ka: area
 * constant (Eq. 14).  mass_total: membrane mass, spread evenly over the nodes
 * (Sec. 2.3.2).  It must be > 0 (it is unused by the Kinematic scheme).
 * Errors: EINVAL (n < 3, n_ks not 1 or n, clockwise order, non-finite input, a
 * node outside 3 <= y <= ny - 4 when walls are present, mass <= 0, ks < 0),
 * ECAPACITY (capsule or node capacity, n > max_nodes_capsule, initial patch too large),
 * ESTATE (after the first step). *capsule_id receives the index (0, 1, ...). */
lbib_status lbib_add_capsule(lbib_ctx* ctx, const double* nodes_xy, int32_t n, const double* ks,
                             int32_t n_ks, double kb, double ka, double mass_total,
                             int32_t* capsule_id);

/* Adds a rigid particle (Sec. 2.3.1) to lattice `lattice`: nodes_xy [n][2]
 * FP64 counter-clockwise outline; mass and moment of inertia about its area
 * centroid (the caller's choice, e.g. (rho_s/rho_f) times the area and the
 * polar second moment of area).  The nodes are driven towards the rigid-body
 * velocity u + omega x r by direct forcing (Dynamic steps 1-3, spreading with
 * c_v = arc length); force and torque come from the stresses at the outer
 * probes x_c + 1.2 n+ (Eqs. 17-18) plus any contact forces on the nodes; the
 * velocities follow Eqs. 19-20; (reading: the paper prints no position
 * update) X += u dt, theta += omega dt, and the nodes are placed at
 * X + R(theta) r0.  Start-up (reading): u and omega are the mean and the
 * least-squares rotation of the interpolated fluid velocity at the nodes.
 * Dynamic scheme only: EINVAL from lbib_step in KINEMATIC mode.  Checks and
 * errors as for lbib_add_capsule_to, plus EINVAL for inertia <= 0. */
lbib_status lbib_add_rigid_to(lbib_ctx* ctx, int32_t lattice, const double* nodes_xy, int32_t n,
                              double mass, double inertia, int32_t* capsule_id);

/* Queues nsteps >= 0 time steps of the chosen scheme on the bound stream.
 * Each step is one IB kernel launch (node update of the previous step fused
 * with the forcing of this step) and one fused collide-stream kernel launch.
 * The call ends with the node update of the last step, so between calls the
 * state is the complete state at time n.
 * Overlapped schedule (lbib_set_overlap): lattices periodic in x (one, or
 * every lattice of a batch) with 1..4096 capsules and no contact force can
 * split the collide-stream pass.  A
 * near kernel covers each capsule's near region (the bounding box of its
 * nodes at n-1 and n plus 5 cells) on the bound stream, and the next IB launch
 * follows it there; a far kernel covers the rest on a second stream of the
 * library's own, so the IB work runs beside it.  The results are
 * bit-identical to the single pass, and the call still returns with all work
 * ordered on the bound stream.  By default the split is used for a single
 * lattice of 2^22 cells or more, where it pays; a batch takes it only when
 * asked (many small lattices: the far launch slows the IB launch beside it
 * more than the split saves).
 * Captured steps (lbib_set_graph(ctx, 1)): otherwise, unless kernel timing is
 * on, the inner steps of a call go in blocks of 16 steps captured once into a
 * HIP graph (one for blocks that start on an even step, one for odd) and
 * replayed with one launch per block; the first step of a call and the
 * remainder launch directly.  The graphs hold kernel launches only and are
 * captured again after the capsule count, the contact cutoff, the mode or the
 * batched pass's tile shape changed.
 * Replays run the very launches of the direct path (bit-identical results).
 * Errors: EINVAL (nsteps < 0, bad mode), ESTATE (mode differs from the first
 * step's), EDEVICE.  Device-side problems raise status flags (lbib_check). */
lbib_status lbib_step(lbib_ctx* ctx, int32_t nsteps, lbib_mode mode);

/* Copies state `what` into dst (dst_bytes long).  capsule_id selects the capsule
 * for LBIB_C_* and the lattice for LBIB_F_* (always 0 for a context made by
 * lbib_create).  dst_is_device = 1: dst is device memory and the copy is queued;
 * 0: host memory and the call waits for the stream.  Errors: EINVAL (unknown
 * what, bad capsule id, dst too small), EDEVICE. */
lbib_status lbib_get_state(lbib_ctx* ctx, int32_t what, int32_t capsule_id, void* dst,
                           size_t dst_bytes, int32_t dst_is_device);

/* Overwrites state `what` (LBIB_F_POPS or LBIB_C_STATE) from src; capsule_id
 * selects as for lbib_get_state.  F_POPS replaces f^n.  The wall populations that Zou-He determines are recomputed.  C_STATE sets
 * x^n, x^{n-1}, u_v^n of one capsule and marks it started.  The stress-free shape
 * is unchanged.  Errors: EINVAL, EDEVICE. */
lbib_status lbib_set_state(lbib_ctx* ctx, int32_t what, int32_t capsule_id, const void* src,
                           size_t src_bytes, int32_t src_is_device);

/* Waits for the stream and reads the device status word.  Returns LBIB_OK if it
 * is clear, LBIB_ENUMERIC otherwise.  The flags are written to *flags_out if it
 * is not NULL.  The word is not cleared. */
lbib_status lbib_check(lbib_ctx* ctx, int32_t* flags_out);

/* Timing of the kernels with HIP events on the stream each runs on.  enable = 1
 * starts recording an event before and after every kernel of lbib_step,
 * enable = 0 stops.  lbib_get_timing waits for the stream and returns
 * out[6] = {grid (or far) kernel total ms, its launches, IB kernel total ms,
 * IB launches, near kernel total ms, near launches}.  It then resets the
 * counters. */
lbib_status lbib_set_timing(lbib_ctx* ctx, int32_t enable);

/* Contact force between capsules (Sec. 3.4, Eq. 27).  cutoff > 0 switches it
 * on: a node at distance d < cutoff (lattice units) from a node of another
 * capsule of the same lattice receives (1e-4 / (8 sqrt 2)) sqrt(1 / d^5) along
 * its inward normal (minus the normalized sum of the outward normals of its
 * two elements), summed over such nodes, nearest periodic image.  The paper
 * gives no cutoff; 2 is the reading the workloads use.  cutoff = 0 (the
 * default) switches it off.  The force joins the total nodal force of the
 * Dynamic update (step 7) and the internal force of the Kinematic forcing
 * (step i), at the positions those use.  Contacts cost one bounds and one
 * contact kernel per force evaluation; the Kinematic scheme then takes
 * separate launches for the node update and the forcing.
 * Errors: EINVAL (cutoff not in [0, 16]), EDEVICE. */
lbib_status lbib_set_contact(lbib_ctx* ctx, double cutoff);

/* Schedule of lbib_step: enable = 1 always uses the overlapped near / far
 * schedule where it applies (see lbib_step), 0 never, -1 (the default) for
 * one lattice of 2^22 cells or more.  In the overlapped schedule of one
 * lattice of 2^23 cells or more, the far kernel of every step after a call's
 * first waits for that step's IB launch on the device (a counter the IB blocks
 * raise), not on the queue; this needs the two streams' kernels to run
 * concurrently.  enable = 2 is the overlapped schedule with queue-level waits
 * only, for tools that run kernels one at a time (counter collection, kernel
 * serialisation): under such a tool the device-side wait gives up after about
 * 0.05 s per block and raises LBIB_FLAG_SYNC.  Results are the same bits in
 * every schedule.  Errors: EINVAL (other values). */
lbib_status lbib_set_overlap(lbib_ctx* ctx, int32_t enable);

/* Membrane checks of the force pass (Eqs. 11-14, evaluated at every step's
 * internal forces): max_edge > 0 raises LBIB_FLAG_EDGE when an element grows
 * longer than max_edge lattice units (Sec. 3.2 keeps the element length below
 * the lattice spacing, or the direct forcing may leave holes in the membrane:
 * max_edge = 1); max_area_change > 0 raises LBIB_FLAG_AREA when the enclosed
 * area leaves A0 by more than that fraction (the penalty of Eq. 14 holds it
 * close).  0 switches a check off; both are off by default.  The flags report
 * and stop nothing.  Errors: EINVAL (negative or non-finite values). */
lbib_status lbib_set_limits(lbib_ctx* ctx, double max_edge, double max_area_change);

/* Captured step blocks of lbib_step: enable = 1 replays them; 0 and -1 (the
 * default, automatic) launch every step directly (on MI355X the replays
 * measure no faster: the direct dispatch keeps pace with these kernels).
 * Errors: EINVAL (other values). */
lbib_status lbib_set_graph(lbib_ctx* ctx, int32_t enable);

/* Number of captured-block replays lbib_step has queued on this context, or
 * -1 for a NULL context. */
int64_t lbib_graph_replays(const lbib_ctx* ctx);

/* Tile shape of the batched grid pass of a batch context (more than one
 * lattice).  rows = nodes per thread (1, 2 or 4): a block of 4 wavefronts
 * covers a 64-cell segment of a band of 4 * rows rows.  linear = the tile
 * order: 0 deals each lattice's bands to the 8 XCDs in groups of 8 (a band and
 * its x-neighbours stay in one XCD's L2; bands padded to a multiple of 8);
 * 1 orders the tiles band by band, segment by segment (no band padding);
 * 2 cuts that linear order into 8 runs of consecutive tiles, one per XCD (a
 * tile's x- and y-neighbours mostly in the same L2; no band padding).  resident = 0
 * launches one block per tile; k in 1..64 launches k blocks per compute unit
 * (rounded to a multiple of 8) that loop over the tiles (a persistent launch).
 * Every shape computes the same bits.  The default is rows 1, linear 0,
 * resident 0.  Errors: EINVAL (other values). */
lbib_status lbib_set_tile(lbib_ctx* ctx, int32_t rows, int32_t linear, int32_t resident);

/* Autotuner of the batched grid pass: times every tile shape (rows 1, 2, 4 with
 * linear 0, then with linear 1, then with linear 2; each with resident 0, 2, 4,
 * 8: out_us[4 * shape + resident index], 36 values) over `launches` grid passes
 * each on the context's own lattices and current state, with HIP events on
 * the bound stream, and keeps the fastest for lbib_step.  The trial passes
 * read no IB force and leave the state unchanged (they write only the
 * population buffer the next step overwrites).  Call it between lbib_step
 * calls.  Outputs (host, each may be NULL): the chosen rows, tile order and
 * resident count, and up to n_us of the mean times per pass in us.  Waits for
 * the stream.  Errors: EINVAL (single-lattice context, launches not in
 * [1, 1000]), EDEVICE. */
lbib_status lbib_autotune(lbib_ctx* ctx, int32_t launches, int32_t* out_rows, int32_t* out_linear,
                          int32_t* out_resident, double* out_us, int32_t n_us);
lbib_status lbib_get_timing(lbib_ctx* ctx, double* out6);

/* Number of completed steps n, or -1 for a NULL context. */
int64_t lbib_steps_done(const lbib_ctx* ctx);

/* Last error message of ctx (or of the calling thread when ctx is NULL). */
const char* lbib_last_error(const lbib_ctx* ctx);

/* ---- Ensembles: many independent lattices in one context ----
 *
 * A batch context holds n_inst independent simulations of the method
 * (Secs. 2.1-2.4 each), every one with its own lattice size, tau, walls and
 * capsules.  They share the eight buffers (each lattice's arrays follow the
 * previous lattice's) and step in lockstep: one lbib_step queues, per time
 * step, one IB launch over the capsules of all lattices and one grid launch
 * over the cells of all lattices, instead of two launches per simulation.
 * Results are bit-identical to stepping each lattice in a context of its own.
 *  - All lattices share real_bytes and the coupling mode.
 *  - Capacities are per lattice (each lbib_grid's max_capsules and
 *    max_nodes_total); the largest max_nodes_capsule sets the on-chip budget.
 *  - Capsule ids count over the whole context, in the order of
 *    lbib_add_capsule_to calls.
 *  - For the field states (LBIB_F_*), capsule_id of get/set names the lattice.
 *  - One device status word serves the whole batch.
 *  - A context from lbib_create is the batch of one lattice; lbib_add_capsule
 *    is lbib_add_capsule_to lattice 0. */

/* Size of buffer `buffer_id` for the lattices grids[0..n_inst-1], or 0 if any
 * grid is invalid, real_bytes differ, or the totals exceed the supported range
 * (2^20 capsules, 2^26 nodes, 1 <= n_inst <= 65536). */
size_t lbib_required_bytes_batch(const lbib_grid* grids, int32_t n_inst, int32_t buffer_id);

/* Creates a batch context: lattice i has grids[i], relaxation time taus[i] and
 * walls[i] (host arrays of n_inst entries, copied).  Buffers, stream, errors
 * and queued initialisation as for lbib_create, applied to every lattice;
 * EINVAL also if real_bytes differ between lattices or n_inst is out of range.
 * The call waits for the stream before it returns. */
lbib_status lbib_create_batch(const lbib_grid* grids, const double* taus,
                              const lbib_walls* walls, int32_t n_inst,
                              void* const* device_buffers, int32_t n_buffers, void* hip_stream,
                              lbib_ctx** out);

/* lbib_add_capsule into lattice `lattice` (0 <= lattice < n_inst, else
 * EINVAL); the node-range check uses that lattice's ny and walls. */
lbib_status lbib_add_capsule_to(lbib_ctx* ctx, int32_t lattice, const double* nodes_xy, int32_t n,
                                const double* ks, int32_t n_ks, double kb, double ka,
                                double mass_total, int32_t* capsule_id);

/* Number of lattices of the context, or -1 for a NULL context. */
int32_t lbib_num_lattices(const lbib_ctx* ctx);

/* ---- Reverse-mode gradients (adjoint) ----
 *
 * Objectives of the final capsule shape (Sec. 3 diagnostics, FP64). */
enum lbib_objective {
    LBIB_OBJ_TAYLOR = 0,     /* Taylor deformation D of the equivalent ellipse (LBIB_D_TAYLOR) */
    LBIB_OBJ_CENTROID_Y = 1  /* area-centroid height y_c (LBIB_D_CY) */
};

/* Workspace bytes lbib_adjoint needs for nsteps steps of this context with
 * the given checkpoint interval, or 0 if the context is not a single lattice,
 * nsteps < 1 or checkpoint_every < 0.
 *   checkpoint_every == 0 or >= nsteps: the whole forward trajectory is taped
 *     (populations, IB force field and node state of every time level: about
 *     (36 + 16) B per cell per step in FP32, linear in nsteps).
 *   0 < checkpoint_every = K < nsteps: the grid state is kept at every K-th
 *     level only (ceil(nsteps / K) checkpoints) plus a tape of K + 1 levels
 *     that the reverse sweep refills segment by segment; the node state of
 *     every level, with the force each node spread, is still taped (a few kB
 *     per level). */
size_t lbib_adjoint_bytes(const lbib_ctx* ctx, int32_t nsteps, int32_t checkpoint_every);

/* Runs nsteps time steps of the chosen scheme from the initial state (the
 * context must be at step 0), taping the trajectory into `workspace` (device
 * memory, caller-owned, lbib_adjoint_bytes(ctx, nsteps, checkpoint_every)
 * long), evaluates J = objective(capsule) at step nsteps, then runs the reverse
 * sweep: the exact discrete adjoint of the executed step (Secs. 2.1-2.4), one
 * reverse grid launch and one reverse IB launch per step.  With a checkpoint
 * interval K (0 < K < nsteps) the reverse sweep goes segment by segment, last
 * first: it restores the segment's checkpoint and runs its K grid steps
 * again into the short tape, each fed by the force level that the taped node
 * forces spread (the same fixed-point contributions as the first run, so the
 * recomputed levels repeat it bit for bit), then reverses them.  J and the
 * final state equal those of the full tape exactly; the gradients equal them
 * up to the summation order of the reverse IB kernel's floating-point
 * atomics (which also varies between two full-tape runs).  The price is one
 * more pass of grid steps and light spreading launches.
 * Outputs (host):
 *   *out_J       J
 *   *out_dJ_dg   dJ/dg for the uniform body force g (the walls' body_force_x),
 *                including its use in the initial Poiseuille profile
 *                (init_profile 2)
 *   out_dJ_dks   dJ/dk_s for every element of every capsule, in node order
 *                (capsule after capsule, element l joins node l to l+1);
 *                n_ks >= total node count
 * Afterwards the context stands at step nsteps, as after lbib_step(nsteps).
 * The MLS supports are held fixed (they are piecewise constant in the
 * positions); the fixed-point rounding of the spread force is not
 * differentiated.
 * Errors: EINVAL (batch context, nsteps < 1, checkpoint_every < 0, bad mode,
 * objective or capsule id, a rigid particle, the contact force on, an open
 * channel, workspace or n_ks too small, NULL pointers), ESTATE (context not at step 0, or its mode differs), ECAPACITY
 * (capsules too large for the on-chip memory of the reverse IB kernel),
 * ENUMERIC (a device status flag in the forward run or the reverse sweep),
 * EDEVICE.  Waits for the stream. */
lbib_status lbib_adjoint(lbib_ctx* ctx, int32_t nsteps, int32_t checkpoint_every, lbib_mode mode,
                         int32_t objective, int32_t capsule, void* workspace,
                         size_t workspace_bytes, double* out_J, double* out_dJ_dg,
                         double* out_dJ_dks, int32_t n_ks);

/* ---- Gradient without allocation ----
 *
 * For callers that cannot allocate device memory: code being captured into a
 * HIP graph, tight serving loops, harnesses that forbid hipMalloc.  Same
 * computation, arguments, outputs and errors as lbib_adjoint, without the
 * workspace argument: the workspace is a static device array of
 * LBIB_ADJOINT_SCRATCH_BYTES (64 MiB) inside the library, one copy on each
 * GPU the library runs on, held until the process ends.  This call allocates
 * nothing (no hipMalloc, no allocating library routine).  It fits gradients
 * whose lbib_adjoint_bytes(ctx, nsteps, checkpoint_every) is at most that size:
 * small lattices, short runs, or a checkpoint interval.
 * Additional errors: ECAPACITY if the workspace would exceed
 * LBIB_ADJOINT_SCRATCH_BYTES (checked before anything is launched); EDEVICE
 * if the context's device is not the current one.
 * Sharing: every call on one GPU uses the same array and leaves its contents
 * behind; each call clears the bytes it uses before the forward run.  Calls
 * that overlap in time on one GPU (several threads or streams) race on the
 * array and give wrong results.  Waits for the stream. */
#define LBIB_ADJOINT_SCRATCH_BYTES (64u * 1024u * 1024u)
lbib_status lbib_adjoint_noalloc(lbib_ctx* ctx, int32_t nsteps, int32_t checkpoint_every,
                                 lbib_mode mode, int32_t objective, int32_t capsule,
                                 double* out_J, double* out_dJ_dg, double* out_dJ_dks,
                                 int32_t n_ks);

/* Frees the host-side context.  Device buffers stay with the caller.  Waits for
 * the stream first. */
void lbib_destroy(lbib_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBIB_H */

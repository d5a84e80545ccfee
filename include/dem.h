/*
 * dem.h -- C ABI of libdem, an MI355X (gfx950) implementation of the
 * rounded-polytope Discrete Element Method for molecular dynamics of
 * Spellings, Marson, Anderson & Glotzer (arXiv:1607.02427).
 *
 * One handle is one periodic system of N rigid rounded polygons (2D) or
 * polyhedra (3D).  Per time step the library computes, on the GPU:
 *   - a cell list and a full neighbour list, rebuilt when a particle has
 *     moved more than rebuild_frac * skin since the last build;
 *   - pair forces, torques, energies and virials by Eq. 1 (3D: every
 *     edge-edge and vertex-face feature pair, Sec. II) or Eq. 2 (2D: every
 *     vertex-edge pair), each evaluated at the features' nearest points under
 *     the WCA potential of Eq. 3-4 with sigma_ij = r_i + r_j;
 *   - a second-order rigid-body integrator (Sec. IV.A) with an optional
 *     Nose-Hoover thermostat on translation and rotation (Sec. IV.C).
 *
 * Conventions
 *   - Units are reduced (m, epsilon, tau; Sec. IV.A).
 *   - All device pointers are HIP device addresses on the current device.
 *   - Every call is asynchronous on the stream given at creation, except
 *     dem_energy, dem_sync, dem_copy_lists and dem_force_stats, which
 *     synchronise that stream.
 *   - Errors: every call returns a dem_status.  Device-side conditions
 *     (neighbour-row overflow and cell overflow: DEM_E_CAPACITY; non-finite
 *     position or velocity: DEM_E_NONFINITE) are latched on the device and
 *     reported by every later synchronising call (dem_sync, dem_energy,
 *     dem_batch_progress) until dem_set_state replaces the state;
 *     dem_last_error gives text.
 *   - Ownership: state and output arrays belong to the caller, which keeps
 *     them alive and unmoved for the handle's lifetime.  Shape and parameter
 *     structs are copied at creation.  Lists, cells and reduction scratch
 *     belong to the library and are freed by dem_destroy_system.
 */
#ifndef DEM_H
#define DEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dem_system *dem_handle;

typedef enum {
    DEM_OK = 0,
    DEM_E_ARG = 1,       /* invalid argument or inconsistent parameters */
    DEM_E_SHAPE = 2,     /* shape tables fail validation or exceed limits */
    DEM_E_OOM = 3,       /* device allocation failed */
    DEM_E_HIP = 4,       /* a HIP runtime call failed */
    DEM_E_CAPACITY = 5,  /* a neighbour row overflowed nbr_capacity, or a cell its 64 slots */
    DEM_E_NONFINITE = 6, /* a position or velocity became non-finite */
    DEM_E_STATE = 7      /* handle in an unusable state */
} dem_status;

enum { DEM_FP64 = 0, DEM_FP32 = 1 };  /* pair-geometry precision */
enum { DEM_NVE = 0, DEM_NVT = 1, DEM_NPT = 2 };
/* List build selector.  Both values take the same device-wide build (cells,
 * then a neighbour scan of 16 lanes per particle, then the pair list), so
 * the lists are the same; the field is kept so parameter blocks stay
 * valid. */
enum { DEM_LISTS_AUTO = 0, DEM_LISTS_MULTI = 1 };

/* Limits of one shape (vertices, edges, faces, face-loop entries) and of the
 * number of shapes per system. */
enum { DEM_MAX_VERTS = 16, DEM_MAX_EDGES = 32, DEM_MAX_FACES = 20, DEM_MAX_LOOP = 64, DEM_MAX_SHAPES = 4 };

/* One rigid shape (Sec. II, Fig. 1): body-frame feature tables.  The body
 * frame is the principal frame with its origin at the centre of mass.
 * 2D: vertices counter-clockwise with z = 0; edge k = (k, k+1 mod n) (Sec.
 * III: the edge beginning at a vertex, travelling counter-clockwise).
 * 3D: faces are planar vertex loops, counter-clockwise seen from outside,
 * convex or concave (Fig. 1a); every edge must appear in the edge table.
 * A single vertex at the origin with no edges and no faces is a sphere (2D:
 * a disk) of radius rounding_radius (edges and face tables may then be
 * null): two of them interact by the central WCA potential of Eq. 3/4 at
 * the distance of their centres, the spheres of Sec. IV.B; against a
 * polytope the point enters Eq. 1/2 as one vertex. */
typedef struct {
    int32_t dim;                  /* 2 or 3, equal to the system's */
    int32_t n_vertices;
    const double *vertices;       /* [n_vertices][3] */
    int32_t n_edges;
    const int32_t *edges;         /* [n_edges][2] vertex indices */
    int32_t n_faces;              /* 0 in 2D */
    const int32_t *face_offsets;  /* [n_faces+1] into face_vertices */
    const int32_t *face_vertices; /* loop vertex indices */
    double rounding_radius;       /* r: surface at r from the features; sigma_ij = r_i + r_j */
    double mass;
    double inertia[3];            /* principal moments; 2D uses inertia[2] */
} dem_shape_desc;

typedef struct {
    int32_t dim;                  /* 2 or 3 */
    int64_t n;                    /* particles, >= 0 */
    double box[3];                /* periodic orthorhombic box; 2D ignores box[2] */
    int32_t n_shapes;             /* 1..DEM_MAX_SHAPES */
    const dem_shape_desc *shapes;
    double epsilon;               /* WCA energy scale (Eq. 3) */
    double skin;                  /* neighbour-list skin */
    double rebuild_frac;          /* rebuild when max displacement > rebuild_frac * skin */
    double dt;
    int32_t ensemble;             /* DEM_NVE, DEM_NVT or DEM_NPT */
    double kT;                    /* thermostat temperature (NVT, NPT) */
    double tau_T;                 /* thermostat time constant: Q = g kT tau_T^2 */
    int32_t precision;            /* DEM_FP64 or DEM_FP32 */
    double parallel_sin2;         /* edges with |u x v|^2 < parallel_sin2 |u|^2 |v|^2
                                     use the overlap-midpoint rule (Sec. II) */
    int32_t nbr_capacity;         /* neighbour-row capacity; 0 = automatic */
    int32_t list_mode;            /* DEM_LISTS_AUTO or DEM_LISTS_MULTI */
    double pressure;              /* DEM_NPT: target pressure P (>= 0) */
    double tau_P;                 /* DEM_NPT: barostat time constant, W = (N_f + d) kT tau_P^2 */
} dem_params;

/* Caller-owned device arrays, FP64 structure-of-arrays, length n, borrowed
 * for the handle's lifetime.  q is the unit quaternion (w, x, y, z) mapping
 * body to space; L is the angular momentum in the body frame; image holds
 * periodic image counters [n][3].  Positions must lie in [0, box). */
typedef struct {
    double *x, *y, *z;
    double *qw, *qx, *qy, *qz;
    double *vx, *vy, *vz;
    double *Lx, *Ly, *Lz;
    int32_t *shape_id;
    int32_t *image;
} dem_state_ptrs;

/* Caller-owned device outputs, FP64, written by dem_compute_forces and every
 * step: force, torque about the centre (space frame; 2D uses Tz), per-particle
 * energy U_i = 1/2 sum_j U_ij and virial W_i = 1/2 sum_j (x_i - x_j) (x) F_ij
 * stored component-major: W[(3a + b) * n + i]. */
typedef struct {
    double *Fx, *Fy, *Fz;
    double *Tx, *Ty, *Tz;
    double *U;
    double *W;                    /* [9][n] */
} dem_output_ptrs;

typedef struct {
    double U, K_trans, K_rot;
    double H;                     /* K + U (NVE); K + U + Q xi^2/2 + g kT eta (NVT); NPT adds
                                     W v_eps^2/2 + P V, with g and Q counting the barostat */
    double T;                     /* 2K / g (g without the barostat's degree of freedom) */
    double P;                     /* (2 K_trans + tr W) / (d V) */
    double W[9];                  /* sum_i W_i */
    double xi, eta;               /* thermostat variables */
    int64_t step;
    int64_t n_rebuilds;
    double V;                     /* box volume (area in 2D) */
    double box[3];                /* current box (it changes under DEM_NPT) */
    double veps;                  /* barostat velocity v_eps (DEM_NPT), d ln V / dt = d v_eps */
} dem_energy_out;

/* Creates a system on the current device and stream, validates and uploads
 * the shape tables, allocates lists, builds them and computes the forces of
 * the initial state.  On error *out is NULL. */
dem_status dem_create_system(const dem_params *params, const dem_state_ptrs *state, const dem_output_ptrs *outputs,
                             void *hip_stream, dem_handle *out);

/* Frees library-owned device memory and the handle (synchronises). */
dem_status dem_destroy_system(dem_handle h);

/* Rebuilds the cell list and the neighbour list from the current positions
 * (cell size L / floor(L / r_list), r_list = 2 R_max + 2^(1/6) sigma_max +
 * skin).  Synchronises; grows the row capacity and rebuilds if a row
 * overflowed and the capacity is automatic. */
dem_status dem_build_celllist(dem_handle h);

/* Computes F, tau, U_i and W_i for the current positions and orientations
 * over the current neighbour list (Eq. 1 / Eq. 2 with Eq. 4). */
dem_status dem_compute_forces(dem_handle h);

/* Advances n_steps time steps (lists rebuilt on the displacement trigger).
 * With NVT the thermostat half steps that fall between two steps are
 * carried across calls: dem_step(a) then dem_step(b) gives the same numbers,
 * bit for bit, as dem_step(a + b).  On return the velocities, L and the
 * reported xi, eta are those at the end of the last step. */
dem_status dem_step(dem_handle h, int64_t n_steps);

/* dem_step under the batch name: on a batch handle every live replica
 * advances up to n_steps steps, each stopping at its own step budget. */
dem_status dem_batch_step(dem_handle h, int64_t n_steps);

/* Where the handle's results live on the device: the force outputs (for a
 * single system the caller's own arrays; for a batch its internal ones,
 * replica r at particle slots [offset, offset + n) of dem_batch_info) with
 * the virial's stride (W[c * w_stride + i]), and the neighbour rows,
 * library-owned: nbr[k * nbr_stride + i] for k < n_nbr[i], ascending, at
 * most capacity per row.  The addresses stay valid until a call changes the
 * row capacity or destroys the handle. */
typedef struct {
    const double *Fx, *Fy, *Fz, *Tx, *Ty, *Tz, *U, *W;
    int64_t w_stride;
    const int32_t *nbr, *n_nbr;
    int64_t nbr_stride;
    int32_t capacity;
} dem_output_view;
dem_status dem_get_outputs(dem_handle h, dem_output_view *out);

/* Checkpoint of a single system (the whole state and the thermostat, so a
 * run resumed from it continues bit for bit as the original would have).
 * dem_state_bytes gives the buffer size (0 for a batch handle or a null
 * handle).  dem_get_state synchronises and writes the checkpoint to a host
 * buffer of at least that size; dem_set_state reads one back (same
 * dimension and particle count), rebuilds the lists, recomputes the forces
 * and clears latched device errors.  DEM_E_ARG for a short buffer, a
 * foreign or mismatched checkpoint or a batch handle (whose replicas are
 * saved with dem_batch_read and restored with dem_batch_add). */
size_t dem_state_bytes(dem_handle h);
dem_status dem_get_state(dem_handle h, void *host_buf, size_t bytes);
dem_status dem_set_state(dem_handle h, const void *host_buf, size_t bytes);

/* Reduces energies, kinetic terms, virial and thermostat state in FP64 and
 * reports latched device errors.  Synchronises. */
dem_status dem_energy(dem_handle h, dem_energy_out *out);

/* Synchronises and reports latched device errors. */
dem_status dem_sync(dem_handle h);

/* Sets the Nose-Hoover variables (for checkpoint/restore); the next step
 * opens its half step from the current kinetic energy. */
dem_status dem_set_thermostat(dem_handle h, double xi, double eta);

/* Sets the barostat velocity v_eps of a DEM_NPT system (Sec. IV.C; a stored
 * state's), after dem_set_thermostat if both are set; the next step opens
 * its half steps from it.  DEM_E_ARG for other ensembles. */
dem_status dem_set_barostat(dem_handle h, double veps);

/* Copies the lists to host buffers (synchronises): cell_start[n_cells+1],
 * cell_particles[n], nbr[capacity * n] column-major (row i of particle i is
 * nbr[k * n + i], k < n_nbr[i], ascending in j) and n_nbr[n].  Any pointer
 * may be NULL.  dims receives {cells_x, cells_y, cells_z, capacity}. */
dem_status dem_copy_lists(dem_handle h, int32_t *cell_start, int32_t *cell_particles, int32_t *nbr, int32_t *n_nbr,
                          int32_t *dims);

/* Neighbour-list radius and number of cells. */
dem_status dem_list_info(dem_handle h, double *r_list, int32_t *n_cells, int32_t *capacity);

/* Work counters accumulated by counted force evaluations since the last
 * reset (out must hold 9 entries): out[0] unordered particle pairs within
 * R_i + R_j + r_cut, out[1] feature-pair problems of Eq. 1/2 left after the
 * per-pair feature prefilter, out[2] feature pairs inside the cutoff,
 * out[3] counted launches, out[4] vertex-face (2D: vertex-edge) problems
 * that pass the per-problem cull and are solved exactly, out[5] FP32
 * feature pairs redone in FP64, out[6] edge-edge problems solved exactly,
 * out[7] pairs of out[0] that a supporting plane of one body separates from
 * the other by more than r_cut (no feature work), out[8] vertex-plane
 * tests made for that separation test.
 * reset != 0 clears them after reading.  Synchronises. */
dem_status dem_force_stats(dem_handle h, int64_t *out, int32_t reset);

/* Enables (on != 0) or disables the work counters inside dem_step's
 * captured step (dem_compute_forces always counts).  Counting adds a few
 * atomics per wave; the arithmetic and results are unchanged. */
dem_status dem_set_counting(dem_handle h, int32_t on);

/* Launches the force kernel alone `reps` times on the current state (no
 * list work, no counters): the launches are captured in one HIP graph, which
 * runs once to warm up and once bracketed by HIP events recorded on the
 * system's stream, and the mean duration of one launch in milliseconds is
 * returned (back-to-back launches, as inside a step graph).  Outputs are
 * overwritten with the same values.  Synchronises. */
dem_status dem_time_forces(dem_handle h, int32_t reps, double *mean_ms);

/* Pair-kernel launch shape (a tuning knob; results do not depend on it,
 * bit for bit): lanes_per_pair (8 or 16) lanes evaluate one particle pair in
 * the feature stage, so a 64-lane wavefront takes 8 or 4 pairs at a time;
 * the grid holds grid_factor (1 to 4) times as many workgroups as the
 * device keeps resident at once; the kernel is compiled for waves_per_simd
 * (2 or 3) resident wavefronts per SIMD (3 overlaps more memory round
 * trips, 2 gives the compiler more registers); and sep_lanes (4, or 16 with
 * 16 lanes per pair) lanes take one pair in the separation stage, so a
 * wavefront settles 16 or 4 pairs at a time and a tile holds 64 or 16
 * pairs (16 spreads a small system over four times the wavefronts).
 * split (0 or 1, the latter with sep_lanes 4) separates the contact search
 * from the force evaluation, the two-step form Sec. V proposes: a search
 * kernel runs the separation stage alone at 4 wavefronts per SIMD and
 * compacts the pairs no supporting plane separates, per replica, into a
 * buffer as large as the pair entries; a force kernel then gives each
 * wavefront one feature round of those pairs (lanes_per_pair and
 * waves_per_simd apply to it; grid_factor does not).  The default is
 * {16, 1, 2, 4, 0}.  The next dem_step captures its graph again.
 * DEM_E_ARG for other values. */
enum { DEM_PAIR_SHAPES = 16 };
dem_status dem_set_pair_shape(dem_handle h, int32_t lanes_per_pair, int32_t grid_factor, int32_t waves_per_simd,
                              int32_t sep_lanes, int32_t split);

/* Feature search (Sec. V: shape-local spatial structures for the contact
 * point search).  on = 0 (default): the feature stage keeps the vertices,
 * edges and faces that lie within reach of the other body's centre and not
 * wholly beyond one of its supporting planes, and pairs every near vertex
 * with every near face and every near edge with every near edge.  on = 1:
 * each shape carries a grid of cells over its body frame (12 per axis in
 * 3D, 40 in 2D, covering its circumradius plus its reach); a cell lists the
 * shape's faces (2D: edges) within the cutoff of any point in it, and its
 * edges within the cutoff plus the longest half edge of the replica's
 * shapes.  After the prefilter above, a near vertex of the other body keeps
 * only the near faces of the cell it lies in, and a near edge only the near
 * edges of the cell that holds its midpoint.  Both forms keep every feature
 * pair inside the
 * cutoff and compute the same terms (within the FP32 path's rounding:
 * the terms are summed in another order); results do not depend on the
 * pair shape in either.  The cells are built on the host with the shape
 * tables (14 KB per shape).  With cells the pair kernel is compiled for 2
 * wavefronts per SIMD whatever the pair shape asks.  The next dem_step
 * captures its graph again.  DEM_E_ARG for other values. */
dem_status dem_set_feature_cells(dem_handle h, int32_t on);

/* Pair-shape autotuner: times `reps` launches of the pair kernel on the
 * current state for each of the DEM_PAIR_SHAPES shapes {lanes, factor,
 * waves, sep, split} = {16,1,2,4,0}, {8,1,2,4,0}, {16,2,2,4,0}, {8,2,2,4,0},
 * {16,1,3,4,0}, {8,1,3,4,0}, {16,2,3,4,0}, {8,2,3,4,0}, {16,1,2,16,0},
 * {16,2,2,16,0}, {16,1,3,16,0}, {16,2,3,16,0}, {16,1,2,4,1}, {8,1,2,4,1},
 * {16,1,3,4,1}, {8,1,3,4,1} (HIP events on the handle's stream) and keeps
 * the fastest.  Outputs (each may be null): shape[5] receives the chosen
 * {lanes, factor, waves, sep, split}, mean_ms[DEM_PAIR_SHAPES] the mean
 * launch time in ms of every shape (both kernels of a split shape), in
 * that order.  The state and lists are not changed; the records of the
 * pair kernel are overwritten by the next step as always.  Synchronises. */
dem_status dem_tune_pairs(dem_handle h, int32_t reps, int32_t *shape, double *mean_ms);

/* Bytes of device memory the library would allocate for these parameters
 * (lists, cells, scratch), excluding caller-owned state and outputs.  For a
 * replica of a batch this is its share of the batch's arrays, less its state
 * and outputs (16 doubles and 4 ints per particle). */
size_t dem_footprint_bytes(const dem_params *params);

/* ---- Batches of independent replicas ------------------------------------
 * A batch handle holds many independent periodic systems ("replicas") of
 * one dimension and one force precision, of any sizes and shapes, and
 * advances all of them with one launch per kernel per step: the pair
 * kernel walks one list of tiles (64 particle pairs of one replica each)
 * over every replica, the list build runs one workgroup per replica, and
 * the integrator and force gather cover every replica's particles.  A
 * replica's arithmetic does not depend on which other replicas share the
 * batch: its results are the same bit for bit alone, in any mix, and as a
 * single system (dem_create_system).  Replicas may be added and removed
 * between calls; each keeps its state in the batch's own device arrays.
 * The batch calls below are asynchronous on the batch's stream unless
 * noted; dem_step, dem_compute_forces, dem_sync, dem_force_stats,
 * dem_set_counting and dem_time_forces accept a batch handle and act on all
 * live replicas. */
typedef struct {
    int32_t dim;                  /* 2 or 3: every replica's */
    int32_t precision;            /* DEM_FP64 or DEM_FP32: every replica's */
    int32_t max_replicas;         /* replica slots */
    int64_t max_particles;        /* particle slots (replicas take multiples of 64) */
    int64_t max_cells;            /* cell slots (a replica takes its cell count + 1); 0 = particles + 2 per replica */
    int32_t max_shapes;           /* shape-table slots; 0 = DEM_MAX_SHAPES per replica */
    int32_t nbr_capacity;         /* neighbour-row capacity of every replica; 0 = grows as replicas need */
    int64_t hbm_budget_bytes;     /* admission budget: device bytes the live replicas may take; 0 = no limit */
} dem_batch_params;

/* Creates an empty batch; allocates all its device memory.  Synchronises. */
dem_status dem_batch_create(const dem_batch_params *params, void *hip_stream, dem_handle *out);

/* Adds a replica: validates params (dim and precision must match the
 * batch; n <= 65536), copies the state from the caller's device arrays
 * (dem_state_ptrs, borrowed for the call only), builds its lists and
 * computes its forces.  The replica then advances with every dem_step for
 * `steps` steps (0 = without limit) and is held still after that.  Admission
 * by footprint: the replica is charged dem_footprint_bytes(params) plus its
 * state and outputs in the batch (16 doubles and 4 ints per particle slot,
 * slots in runs of 64); returns DEM_E_OOM, with nothing changed, when that
 * would take the live replicas' charge over hbm_budget_bytes, or when no run
 * of free particle, cell or shape slots fits it; DEM_E_CAPACITY when rows
 * overflow a fixed capacity.  Synchronises. */
dem_status dem_batch_add(dem_handle h, const dem_params *params, const dem_state_ptrs *state, int64_t steps,
                         int32_t *replica_id);

/* Removes a replica and frees its slots.  Synchronises. */
dem_status dem_batch_remove(dem_handle h, int32_t replica_id);

/* Copies a replica's state and outputs (either may be NULL, as may any of
 * their arrays) to caller-owned device arrays of its length; W as [9][n]. */
dem_status dem_batch_read(dem_handle h, int32_t replica_id, const dem_state_ptrs *state,
                          const dem_output_ptrs *outputs);

/* Sets the steps a replica has left (0 holds it still). */
dem_status dem_batch_set_steps(dem_handle h, int32_t replica_id, int64_t steps);

/* Steps left and steps done of replica slots 0..count-1 (-1 for free slots;
 * either array may be NULL), and latched device errors.  Synchronises. */
dem_status dem_batch_progress(dem_handle h, int64_t *steps_left, int64_t *steps_done, int32_t count);

/* out[10]: live replicas, replica slots, free particle slots, largest run
 * of free particle slots, free cell slots, free shape slots, row capacity,
 * particle slots, bytes charged to the live replicas, admission budget
 * (0 = no limit). */
dem_status dem_batch_info(dem_handle h, int64_t *out);

/* dem_energy and dem_copy_lists for one replica of a batch (replica 0 is
 * what those calls report).  Synchronise. */
dem_status dem_replica_energy(dem_handle h, int32_t replica_id, dem_energy_out *out);
dem_status dem_replica_lists(dem_handle h, int32_t replica_id, int32_t *cell_start, int32_t *cell_particles,
                             int32_t *nbr, int32_t *n_nbr, int32_t *dims);

/* dem_replica_energy without any allocation, for callers that cannot
 * allocate device memory (tight serving loops, code that must not call
 * hipMalloc or an allocating library routine).  Same arguments, same results
 * bit for bit, same latched errors and the same synchronisation of the
 * handle's stream; the per-chunk partials and their totals go to a static
 * device array of 12 * 4096 + 16 doubles (393 KB) that each device holds
 * until the process ends, instead of the handle's reduction buffers.
 * Limit: replicas of at most 4096 chunks of 64 particles (262,144
 * particles); larger ones return DEM_E_CAPACITY with nothing launched.
 * Every call on one device shares that array: calls that overlap on one
 * device (other host threads, other streams) race and must be serialised
 * by the caller; each call writes its totals whole, so nothing left by an
 * earlier call reaches a later one. */
dem_status dem_replica_energy_noalloc(dem_handle h, int32_t replica_id, dem_energy_out *out);

const char *dem_status_string(dem_status s);
const char *dem_last_error(dem_handle h);

#ifdef __cplusplus
}
#endif

#endif /* DEM_H */

// Internal declarations shared by the libdem translation units: device-side
// shape tables, the per-system parameter block passed to every kernel, and
// the host launchers each .hip file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dem.h"

namespace dem {

// 2^(1/6): the WCA cutoff in units of sigma (Sec. II, Eq. 4).
constexpr double kWcaCut = 1.122462048309373;

// Particles per chunk.  Every replica of a batch starts on a chunk
// boundary, so a wavefront's particles (and a gather block's) belong to one
// replica, and per-chunk partial sums do not depend on the other replicas.
constexpr int kChunk = 64;
// The pair kernel: kPairWaves waves per workgroup; its separation stage
// takes 4 lanes per particle pair and its feature stage 8 or 16
// (BatchParams::pair_lanes, chosen by the pair-shape tuner).  A tile is what
// one workgroup takes at a time (16 pairs per wavefront), and tiles never
// straddle replicas.
// The separation stage takes sep_lanes lanes per pair (4: 16 pairs per
// wavefront; 16: 4 pairs per wavefront, which spreads a small system's
// pairs over four times the wavefronts), so a tile is kPairWaves * 64 /
// sep_lanes pairs.
constexpr int kPairWaves = 4;
constexpr int kDefaultPairLanes = 16;
constexpr int kDefaultPairWaves = 2;
constexpr int kDefaultPairSep = 4;
__host__ __device__ constexpr int pair_tile(int sep_lanes) { return kPairWaves * (64 / sep_lanes); }
// Shape-local feature cells (Sec. V): a uniform grid over each shape's
// body frame, kFcGrid3 cells per axis in 3D (kFcGrid2 in 2D), covering the
// shape's circumradius plus its reach.  Cell c holds .x: the faces (3D) or
// edges (2D) within reach of a vertex of another shape lying in c, and .y
// (3D): the edges within reach of an edge of another shape whose midpoint
// lies in c.  Built on the host, conservatively (the cell's centre
// distance less its half diagonal).
constexpr int kFcGrid3 = 12, kFcGrid2 = 40;
constexpr int kFcCells = kFcGrid2 * kFcGrid2 > kFcGrid3 * kFcGrid3 * kFcGrid3 ? kFcGrid2 * kFcGrid2
                                                                             : kFcGrid3 * kFcGrid3 * kFcGrid3;
// What one launch of the pair kernel does: both stages (fused), or, in the
// split form, the contact search (separation stage, compacting the pairs it
// keeps) and then the contact forces (feature stage on those pairs).
enum PairStage { kFused = 0, kSearchOnly = 1, kForces = 2 };
constexpr int kSearchOcc = 4;  // wavefronts per SIMD of the search kernel

// Per-replica device flag words (flags[r * FLAG_COUNT + w], one 64-byte
// line per replica).  FLAG_TRIGGER: some particle has moved far enough
// since the last build that the next step must rebuild the lists;
// FLAG_REBUILD: the current step rebuilds them (from the positions after
// its drift; the new lists serve from the next step on).  FLAG_NPAIRS: pair
// entries of the lists in use; FLAG_NEWPAIRS: those of the build under way.
// FLAG_FILL: the current step's build writes its pair entries (a copy of
// FLAG_REBUILD taken by the gather, for the extra workgroups of the replica
// tail, while the tail itself moves FLAG_REBUILD on to the next step).
enum Flag {
    FLAG_REBUILD = 0, FLAG_NBUILDS = 1, FLAG_MAXROW = 2, FLAG_NONFINITE = 3, FLAG_NPAIRS = 4,
    FLAG_TRIGGER = 6, FLAG_CELLOVF = 7, FLAG_NEWPAIRS = 9, FLAG_FILL = 10, FLAG_BOXSMALL = 11, FLAG_COUNT = 16
};
// Batch-wide words.  G_ANY: how many replicas rebuild their lists in the
// current step (the list workgroups of the step kernels return at once
// when none does); G_FILL: its copy taken by the gather, for the replica
// tail.  G_STAMP: number of the current force evaluation (bumped before
// every launch of the pair kernel in a step or a force computation).
enum GWord { G_ANY = 0, G_STAMP = 1, G_FILL = 2, G_COUNT = 4 };
// Particles one cell can hold, and the longest neighbour row.
constexpr int kCellCap = 64;
constexpr int kRowMax = 128;
// Particles whose neighbour rows one wavefront builds at a time (16 lanes
// each); the pair counts are totalled per such group (ListPtrs::ptot).
constexpr int lb_rows_per_group = 4;
// Per-replica thermostat words (double, thermo[r * TH_COUNT + w]).  Between
// steps a replica is either closed (its velocities carry every half step
// so far) or open: the closing half step of its last step has scaled the
// thermostat but not yet the velocities (pending factor TH_SB), and the
// opening half step of its next step is computed (pending factor TH_SA;
// TH_XI, TH_ETA after it).  TH_XI_B, TH_ETA_B hold xi and eta at the end of
// the last completed step.  The next kick applies (v * SB) * SA, and the
// end of a call applies SB alone, so a run split into calls and the same
// run in one call give the same numbers.
// DEM_NPT adds the barostat velocity after the opening half step of the
// current step (TH_VEPS) and at the end of the last completed step
// (TH_VEPS_B), and the step's factors of the exact kick and drift flows:
// TH_DAMP = exp(-alpha v_eps h/2), TH_FK = (h/2) exp(-alpha v_eps h/4)
// sinhc(alpha v_eps h/4), TH_GROW = exp(v_eps h), TH_VFAC = h exp(v_eps h/2)
// sinhc(v_eps h/2) (sinhc(u) = sinh(u) / u).
enum Thermo {
    TH_XI = 0, TH_ETA = 1, TH_SB = 2, TH_SA = 3, TH_XI_B = 4, TH_ETA_B = 5, TH_OPEN = 6,
    TH_VEPS = 8, TH_VEPS_B = 9, TH_DAMP = 10, TH_FK = 11, TH_GROW = 12, TH_VFAC = 13, TH_BOXN = 16, TH_COUNT = 24
};
// (TH_BOXN..TH_BOXN + 2: the box of the current positions.  Inside a call
// the replica tail already moves SysParams::box on to the next step's box;
// the end of a call puts the box of the positions back and the next call's
// first step applies TH_GROW again.)
// Per-chunk reduction partials of the step: K_trans, K_rot, tr W, (pad).
constexpr int kKePer = 4;
// Force work counters (unsigned long long).
enum Stat {
    ST_PAIRS = 0, ST_FEATURES = 1, ST_INCUT = 2, ST_LAUNCHES = 3, ST_NEAR = 4, ST_REFINED = 5, ST_EENEAR = 6,
    ST_SEPARATED = 7, ST_PLANETESTS = 8, ST_COUNT = 9
};

// One row-slot record, for slot k of particle i's neighbour row at
// rec[k * N + i]: the force on i (space frame) and the pair energy U_ij,
// the torque on i about its centre, and the pair offset x_j - x_i, each
// padded to a 16-byte word so one record is three (FP64: six) whole
// vector loads.  The force pass writes both slots of a pair.
template <typename T>
struct alignas(16) SlotRec {
    T F[3], U;
    T tq[3], pad0;
    T d[3], pad1;
};
// The first pad word carries the G_STAMP of the force evaluation that wrote
// the record.  The gather adds only records of the current evaluation, so a
// pair with no feature pair inside the cutoff writes nothing at all.
// (Storage starts zeroed: a record never written adds zeros.)
__device__ inline unsigned slot_stamp(const SlotRec<float> &w) { return __float_as_uint(w.pad0); }
__device__ inline unsigned slot_stamp(const SlotRec<double> &w) { return (unsigned)__double_as_longlong(w.pad0); }
__device__ inline void set_stamp(SlotRec<float> &w, unsigned s) { w.pad0 = __uint_as_float(s); }
__device__ inline void set_stamp(SlotRec<double> &w, unsigned s) { w.pad0 = __longlong_as_double((long long)s); }

// Body-frame feature tables of one shape in precision T, staged in LDS.
// Edges carry their vector, midpoint, half length and 1/|edge|^2; faces
// their outward unit normal n and offset o (n.x = o on the plane), a
// bounding circle (centroid, radius), the in-plane inward normal and offset
// of each loop edge (convex inside test), face coordinates of each loop
// vertex (crossing-number test for concave faces) and 1/|loop edge|^2.
// The supporting planes (3D: the face planes with the whole body on their
// inner side; 2D: such edge lines) carry unit normal sn and offset so =
// max over vertices of sn.v, so every point of the inner body satisfies
// sn.x <= so.
constexpr int kMaxSep = DEM_MAX_EDGES > DEM_MAX_FACES ? DEM_MAX_EDGES : DEM_MAX_FACES;
template <typename T>
struct alignas(16) ShapeTab {
    int nv, ne, nf;
    int fc_g;                    // shape-local feature cells: fc_g cells per axis
    T r, R;
    T fc_lo, fc_ih;              // covering [fc_lo, -fc_lo] per axis, 1 / cell width
    T v[DEM_MAX_VERTS][3];
    int e[DEM_MAX_EDGES][2];
    T ed[DEM_MAX_EDGES][3];      // edge vector b - a
    T em[DEM_MAX_EDGES][3];      // edge midpoint
    T eh[DEM_MAX_EDGES];         // half length
    T el2[DEM_MAX_EDGES];        // |b - a|^2
    T einv[DEM_MAX_EDGES];       // 1 / |b - a|^2
    int foff[DEM_MAX_FACES + 1];
    int floop[DEM_MAX_LOOP];
    int fconvex[DEM_MAX_FACES];
    T fn[DEM_MAX_FACES][3];
    T fo[DEM_MAX_FACES];
    T fc[DEM_MAX_FACES][3];      // centroid of the loop vertices
    T frad[DEM_MAX_FACES];       // max distance from fc to a loop vertex
    T fe1[DEM_MAX_FACES][3];     // face axis 1; axis 2 = n x axis 1; origin = first loop vertex
    T lnrm[DEM_MAX_LOOP][3];     // inward in-plane normal of loop edge k -> k+1
    T loff[DEM_MAX_LOOP];        // lnrm . b_k
    T linv[DEM_MAX_LOOP];        // 1 / |b_{k+1} - b_k|^2
    T lxy[DEM_MAX_LOOP][2];      // face coordinates of loop vertex k
    int nsep, pad3[3];
    T sn[kMaxSep][3];            // supporting-plane normals
    T so[kMaxSep];               // and offsets
};

static_assert(sizeof(ShapeTab<float>) % 16 == 0 && sizeof(ShapeTab<double>) % 16 == 0, "tables are copied in 16-byte words");

// One replica: a periodic system of its own.  A single system is a batch
// of one replica.  Indices into batch arrays are global particle slots;
// replica r owns slots [off, off + n), cells [coff, coff + ncell] and pair
// slots [poff, poff + pcap).
struct SysParams {
    int n, dim, n_shapes, live;
    int off;                     // first particle slot (a multiple of kChunk)
    int coff;                    // first cell slot (ncell + 1 entries of cell_start)
    int poff;                    // first pair slot
    int pcap;                    // pair slots
    int sbase;                   // first shape-table slot
    int nc[3], ncell;
    int use_cells;               // 1 if every periodic axis has >= 3 cells
    int ensemble;
    int rid;                     // replica slot
    double box[3];
    double cellw[3];             // box / nc
    double rl2;                  // r_list^2
    double disp2;                // (rebuild_frac * skin)^2
    double eps, par_s2;
    double dt, kT, g, Qm;
    // DEM_NPT (Sec. IV.C): target pressure, barostat mass W = (N_f + d) kT
    // tau_P^2, alpha = 1 + d / N_f with N_f = d (n - 1); the box at the last
    // list build; r_list and the cells per axis at creation.  box, cellw,
    // nc, ncell and use_cells of an NPT replica change on the device every
    // step (the replica tail), and the host reads them back before using them.
    double pext, Wm, alpha;
    double box_build[3];
    double rlist;
    int nc0[3], pad_npt;
    double mass[DEM_MAX_SHAPES];
    double inertia[DEM_MAX_SHAPES][3];
    double R[DEM_MAX_SHAPES];    // circumradius about the body origin
    double rad[DEM_MAX_SHAPES];  // rounding radius
};

// Batch-wide parameters, passed by value to every kernel.
struct BatchParams {
    int nrep;                    // replica slots in use (slots with live == 0 are skipped)
    int N;                       // particle slots: stride of the library's column-major arrays
    int wstride;                 // stride of the virial output W[9][.]
    int nstate;                  // length of the state and output arrays: N for a batch's own
                                 // arrays, n for the arrays a single system borrows
    int nchunk;                  // chunks in use (kernels over particles cover nchunk * kChunk slots)
    int cap;                     // neighbour-row capacity
    int tab_slots;               // shape tables of one replica staged in LDS
    int pair_blocks;             // grid of the pair kernel (a multiple of 8)
    int pair_lanes;              // lanes per particle pair in the pair kernel (8 or 16)
    int pair_waves;              // its wavefronts per SIMD (2 or 3)
    int pair_sep;                // lanes per pair in its separation stage (4 or 16)
    int tile;                    // pairs per tile: pair_tile(pair_sep)
    int pair_split;              // 1: two kernels, contact search then contact forces
    int feature_cells;           // 1: the feature search reads the shape-local feature cells
    int search_blocks;           // grid of the search kernel of the split form
    int dim;
};

struct StatePtrs {
    double *x, *y, *z, *qw, *qx, *qy, *qz, *vx, *vy, *vz, *Lx, *Ly, *Lz;
    int32_t *sid, *image;
};

struct OutPtrs {
    double *Fx, *Fy, *Fz, *Tx, *Ty, *Tz, *U, *W;
};

struct ListPtrs {
    int32_t *cell_count;         // [cells] particles in each cell (zero between builds)
    int32_t *cell_slot;          // [cells][kCellCap] particles of each cell, unordered
    int32_t *pcell;              // [N] cell of each particle, local to its replica
    int32_t *nbr, *n_nbr;        // [cap][N] rows (ascending), [N] row lengths
    double *xlast;               // [3][N] positions at the last build
    int32_t *flags;              // [replica][FLAG_COUNT]
    int32_t *gflags;             // [G_COUNT]
    int32_t *tile_start;         // [nrep + 1] first pair tile of each replica
    const int32_t *chunk_rep;    // [nchunk] replica of each chunk, -1 if free
    // half list of unordered pairs (i < j), rebuilt with the neighbour list
    int32_t *klo;                // [N] first row slot of i holding a j > i
    int32_t *pstart;             // [N] first pair index of i, local to its replica
    int32_t *ptot;               // [N / 4] pairs owned by each group of 4 particles (a row workgroup's)
    int4 *pairs;                 // [pair slots] {i, j, slot of j in i's row, slot of i in j's row (-1: missing)}
    // row slots whose record was written since the particle's last gather:
    // bit k % 32 of word k / 32, [slot_words(cap)][N]; the gather reads
    // only those records and clears the words
    uint32_t *smask;
    // Split form of the pair kernel (contact search, then contact forces):
    // the pairs no supporting plane separates, compacted per replica into
    // its own range of pair slots ([pair slots], order not fixed); their
    // count per replica, the force kernel's first unit of each replica
    // ([nrep + 1]) and two tickets, laid out as split_ctl below.
    int4 *cpairs;
    // shape-local feature cells ([shape slots][kFcCells]; see fc_lookup)
    const uint2 *fcells;
    int32_t *ccount;             // [replica slots] compacted pairs (zero between evaluations)
    int32_t *cunit;              // [replica slots + 1] first force unit of each replica
    int32_t *ctick;              // [2] blocks done: search kernel, force kernel
};
__host__ __device__ inline int slot_words(int cap) { return (cap + 31) / 32; }
// ints of the split form's control words for `replicas` replica slots:
// ccount [replicas], cunit [replicas + 1], ctick [2]
inline size_t split_words(int replicas) { return 2 * (size_t)replicas + 3; }

// Everything the pair kernel reads about one particle, in one cache line:
// FP64 position, the body-to-space rotation in the force precision (row
// major) and the shape id.  Written by the kick-drift (and by
// launch_rotations from the state arrays).
template <typename T>
struct PartRec;
template <>
struct alignas(64) PartRec<float> {
    double x, y, z;
    float R[9];
    int sid;
};
template <>
struct alignas(128) PartRec<double> {
    double x, y, z;
    double R[9];
    int sid;
    int pad[7];
};

// FP64 position and orientation of one particle, for the FP32 pair path's
// FP64 redo of problems FP32 cannot resolve.
struct alignas(64) PartRec64 {
    double x, y, z, qw, qx, qy, qz, pad;
};

struct ForcePtrs {
    void *rot;                   // [N] PartRec<T>
    PartRec64 *rec64;            // [N], FP32 path only (else null)
    void *rec;                   // [cap][N] SlotRec<T> row-slot records
    const void *tab;             // shape tables, precision T
    const void *tab64;           // shape tables, FP64 (refinement of ill-conditioned FP32 problems)
};

// ---- launchers (all asynchronous on `stream`) ----
// `reps` is the device array of replica parameters; `host` the host copy of
// replica 0, used only by the one-kernel-per-phase list build of a single
// large system.
struct Launch {
    BatchParams b;
    const SysParams *reps;
    StatePtrs s;
    OutPtrs o;
    ListPtrs l;
    ForcePtrs f;
    int precision;
    double *ke_part;             // [kKePer * nchunk]
    double *thermo;              // [replica][TH_COUNT]
    int64_t *budget;             // [replica] steps left; a replica with none left is held still
    int64_t *steps;              // [replica] steps done
};

// ---- isothermal-isobaric steps (DEM_NPT, Sec. IV.C) ----------------------
// The barostat follows the measure-preserving isotropic scheme the paper
// cites: dx/dt = v + v_eps x, dv/dt = F/m - (alpha v_eps + xi) v, dV/dt =
// d V v_eps, dv_eps/dt = (alpha 2 K_trans + tr W - d V P) / W - xi v_eps,
// one Nose-Hoover xi for translation, rotation and the barostat.

// sinh(u) / u; its series below |u| = 1e-2 (truncation below 1e-17).
__device__ inline double sinhc(double u)
{
    if (fabs(u) < 1e-2) {
        const double u2 = u * u;
        return 1.0 + u2 * (1.0 / 6.0 + u2 * (1.0 / 120.0 + u2 * (1.0 / 5040.0)));
    }
    return sinh(u) / u;
}

__device__ inline double box_volume(const SysParams &p)
{
    return p.dim == 3 ? p.box[0] * p.box[1] * p.box[2] : p.box[0] * p.box[1];
}

// Thermostat half step of length dt/2 with the barostat's kinetic term in
// its drive; K2 = 2 (K_trans + K_rot) and v_eps are scaled with the
// velocities.  Returns the velocity scale.
__device__ inline double nh_half_npt(const SysParams &p, double &xi, double &eta, double &K2, double &veps)
{
    const double h = 0.5 * p.dt;
    xi += 0.5 * h * (K2 + p.Wm * veps * veps - p.g * p.kT) / p.Qm;
    const double sc = exp(-xi * h);
    K2 *= sc * sc;
    veps *= sc;
    eta += xi * h;
    xi += 0.5 * h * (K2 + p.Wm * veps * veps - p.g * p.kT) / p.Qm;
    return sc;
}

// Barostat half step of length dt/2 from 2 K_trans, tr W and the volume of
// the box in p.
__device__ inline void baro_half(const SysParams &p, double Kt2, double trW, double &veps)
{
    veps += 0.5 * p.dt * (p.alpha * Kt2 + trW - p.dim * box_volume(p) * p.pext) / p.Wm;
}

// The step's kick and drift factors for barostat velocity veps.
__device__ inline void npt_factors(const SysParams &p, double veps, double *th)
{
    const double h = p.dt, a = p.alpha * veps;
    th[TH_DAMP] = exp(-0.5 * h * a);
    th[TH_FK] = 0.5 * h * exp(-0.25 * h * a) * sinhc(0.25 * h * a);
    th[TH_GROW] = exp(h * veps);
    th[TH_VFAC] = h * exp(0.5 * h * veps) * sinhc(0.5 * h * veps);
}

// Sets the box of an NPT replica and its cell geometry: as many cells per
// axis as at creation while they stay at least r_list wide, fewer when the
// box has shrunk; cells are used while every axis has three.  Flags a box
// below twice r_list (the minimum image would no longer be unique).
__device__ inline void set_box(SysParams &p, const double *box, int32_t *fl)
{
    int use = 1, ncell = 1;
    for (int a = 0; a < 3; ++a) {
        p.box[a] = box[a];
        if (a < p.dim) {
            if (box[a] < 2.0 * p.rlist) atomicOr(&fl[FLAG_BOXSMALL], 1);
            const int fit = (int)floor(box[a] / p.rlist);
            p.nc[a] = fit < p.nc0[a] ? (fit > 1 ? fit : 1) : p.nc0[a];
            if (p.nc[a] < 3) use = 0;
        }
        p.cellw[a] = box[a] / (double)p.nc[a];
        ncell *= p.nc[a];
    }
    p.ncell = ncell;
    p.use_cells = use;
}

// Cell list, neighbour list, half pair list and the tile plan of the pair
// kernel, outside a step.  mode LISTS_ALL or a replica index: from the
// current positions, now, for every live replica or for that one (cells
// included).  LISTS_PLAN recomputes the tile plan alone; LISTS_REFILL
// writes every live replica's pair entries again from its rows (after the
// pair slots moved) and the plan.  LISTS_STEP names the build inside a step
// (every replica whose rebuild flag is set and that has steps left), which
// the step kernels carry themselves.
enum { LISTS_STEP = -1, LISTS_ALL = -2, LISTS_PLAN = -3, LISTS_REFILL = -4 };
void launch_lists(const Launch &L, int mode, hipStream_t stream);

// Cell of particle i at (x, y, z), and its insertion into the cell's slots
// (for replicas that use cells).  Bit-exact FP64 binning: the cell is
// min(n_c - 1, floor(x / (L / n_c))) per axis.
__device__ inline void cell_insert(const SysParams &p, const ListPtrs &l, int i, double x, double y, double z)
{
    const double xs[3] = {x, y, z};
    int c3[3] = {0, 0, 0};
    for (int a = 0; a < p.dim; ++a) {
        // clamped before the conversion, so a non-finite position (reported
        // by the kick-drift) still lands in a valid cell: fmax and fmin
        // return the other operand for a NaN
        const double c = fmin(fmax(floor(xs[a] / p.cellw[a]), 0.0), (double)(p.nc[a] - 1));
        c3[a] = (int)c;
    }
    const int c = c3[0] + p.nc[0] * (c3[1] + p.nc[1] * c3[2]);
    l.pcell[i] = c;
    if (!p.use_cells) return;
    const int slot = atomicAdd(&l.cell_count[p.coff + c], 1);
    if (slot < kCellCap) l.cell_slot[(size_t)(p.coff + c) * kCellCap + slot] = i;
    else atomicOr(&l.flags[p.rid * FLAG_COUNT + FLAG_CELLOVF], 1);
}

// Dynamic LDS of the pair kernel, and how many of its blocks the device
// holds at once.
size_t pair_kernel_lds(int precision, int tab_slots, int lanes, int sep, int stage, int fc);
int pair_blocks_resident(int precision, int dim, int tab_slots, int lanes, int waves, int sep, int stage, int fc);

// Per-particle records (position, rotation, shape id) from the state arrays.
void launch_rotations(const Launch &L, hipStream_t stream);

// Pair records over the half lists; stats may be null.
void launch_pairs(const Launch &L, unsigned long long *stats, hipStream_t stream);

// Per-particle sums of pair records in row order (fixed, atomic-free):
// F, tau, U_i, W_i; with kick != 0 also the closing velocity/angular
// momentum kick and then the step tail of every replica (Nose-Hoover half
// steps, step budget and count, rebuild scheduling), which also carries
// the pair entries and the tile plan of the step's list build.
void launch_gather(const Launch &L, bool kick, hipStream_t stream);

// Integrator pieces.  With NVT the step tail after the gather applies the
// closing half step of the step and the opening half step of the next one;
// launch_nh_begin opens the first step of a closed replica,
// launch_nh_end applies the pending closing factor to the velocities.
void launch_nh_begin(const Launch &L, hipStream_t stream);
void launch_kick_drift(const Launch &L, hipStream_t stream);
void launch_kinetic(const Launch &L, hipStream_t stream);
void launch_nh_end(const Launch &L, hipStream_t stream);
// Per-chunk partials of U, K_trans, K_rot and W (9): part[12 * chunk + c].
void launch_energy_partials(const Launch &L, double *part, hipStream_t stream);
void launch_energy_totals(const Launch &L, int c0, int nchunks, double *part, double *total, hipStream_t stream);

constexpr int kBlock = 256;
inline int blocks_for(int n) { return (n + kBlock - 1) / kBlock; }
// Workgroups go to the eight XCDs in turn (block b to XCD b mod 8), each
// with its own L2. A grid of a multiple of 8 blocks read through
// xcd_block() gives XCD x the x-th eighth of the logical blocks, so the
// step kernels (kick and drift, gather) and the pair kernel, which splits
// its tiles the same way, touch a particle's data on the same XCD step
// after step and find it in that L2. Any other grid size keeps the plain
// order (still a permutation, only without the locality).
__host__ __device__ inline int pad8(int blocks) { return (blocks + 7) / 8 * 8; }
__device__ inline int xcd_block(int b, int G) { return (G & 7) ? b : (b & 7) * (G >> 3) + (b >> 3); }
// The gather and the kinetic reduction map one chunk (kGatherPer = kChunk
// particles) to each block of kGatherLanes lanes per particle, which writes
// one kinetic partial.
constexpr int kGatherLanes = 1;
constexpr int kGatherPer = kChunk;
constexpr int kGatherBlock = kChunk * kGatherLanes;

// Rotation matrix (row-major, body to space) of a unit quaternion (w, x, y, z).
__host__ __device__ inline void quat_to_rot(double w, double x, double y, double z, double *R)
{
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

}  // namespace dem

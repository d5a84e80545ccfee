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

// Device flag words.
enum Flag {
    FLAG_REBUILD = 0, FLAG_NBUILDS = 1, FLAG_MAXROW = 2, FLAG_NONFINITE = 3, FLAG_NPAIRS = 4, FLAG_TICKET = 5, FLAG_COUNT = 8
};
// Thermostat words (double): running xi and eta, the velocity scale the next
// kick-drift applies, and the state right after the closing half step of the
// last completed step (xi, eta and its velocity scale).
enum Thermo { TH_XI = 0, TH_ETA = 1, TH_SCALE = 2, TH_XI_B = 3, TH_ETA_B = 4, TH_SCALE_B = 5, TH_COUNT = 8 };
// Force work counters (unsigned long long).
enum Stat {
    ST_PAIRS = 0, ST_FEATURES = 1, ST_INCUT = 2, ST_LAUNCHES = 3, ST_NEAR = 4, ST_REFINED = 5, ST_EENEAR = 6, ST_COUNT = 7
};

// Words of one row-slot record, stored component-major rec[c][k][i] for
// slot k of particle i's neighbour row: force on i (space frame, 3), torque
// on i about its centre (3), pair energy U_ij (1), and the pair offset
// x_j - x_i (3).  The force pass writes both slots of a pair.
constexpr int kRec = 10;

// Body-frame feature tables of one shape in precision T, staged in LDS.
// Edges carry their vector, midpoint, half length and 1/|edge|^2; faces
// their outward unit normal n and offset o (n.x = o on the plane), a
// bounding circle (centroid, radius), the in-plane inward normal and offset
// of each loop edge (convex inside test), face coordinates of each loop
// vertex (crossing-number test for concave faces) and 1/|loop edge|^2.
template <typename T>
struct ShapeTab {
    int nv, ne, nf, pad0;
    T r, R, pad1, pad2;
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
};

// Parameters of one system, passed by value to every kernel.
struct SysParams {
    int n, dim, n_shapes, cap;
    int nc[3], ncell;
    int use_cells;               // 1 if every periodic axis has >= 3 cells
    int ensemble;
    int max_pairs;               // capacity of the pair arrays
    int force_multi_kernel_lists;  // build lists with one kernel per phase even when small
    int pair_blocks;             // grid of the pair kernel (grid-stride over pairs)
    double box[3];
    double cellw[3];             // box / nc
    double rl2;                  // r_list^2
    double disp2;                // (rebuild_frac * skin)^2
    double eps, par_s2;
    double dt, kT, g, Qm;
    double mass[DEM_MAX_SHAPES];
    double inertia[DEM_MAX_SHAPES][3];
    double R[DEM_MAX_SHAPES];    // circumradius about the body origin
    double rad[DEM_MAX_SHAPES];  // rounding radius
};

struct StatePtrs {
    double *x, *y, *z, *qw, *qx, *qy, *qz, *vx, *vy, *vz, *Lx, *Ly, *Lz;
    int32_t *sid, *image;
};

struct OutPtrs {
    double *Fx, *Fy, *Fz, *Tx, *Ty, *Tz, *U, *W;
};

struct ListPtrs {
    int32_t *cell_count, *cell_start, *cell_particles, *pcell, *nbr, *n_nbr;
    double *xlast;               // [3][n]
    int32_t *flags;
    // half list of unordered pairs (i < j), rebuilt with the neighbour list
    int32_t *klo;                // [n] first row slot of i holding a j > i
    int32_t *pstart;             // [n] first pair index of i
    int4 *pairs;                 // [max_pairs] {i, j, slot of j in i's row, slot of i in j's row}
};

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

struct ForcePtrs {
    void *rot;                   // [n] PartRec<T>
    void *rec;                   // [kRec][cap][n] row-slot records, precision T
    const void *tab;             // shape tables, precision T
    const void *tab64;           // shape tables, FP64 (refinement of ill-conditioned FP32 problems)
};

// ---- launchers (all asynchronous on `stream`) ----
// Cell list, neighbour list and half pair list.  The kernels exit at once
// unless the rebuild flag is set, so a captured step contains them
// unconditionally.
void launch_build_lists(const SysParams &p, const StatePtrs &s, const ListPtrs &l, hipStream_t stream);

// Per-particle records (position, rotation, shape id) from the state arrays.
void launch_rotations(const SysParams &p, const StatePtrs &s, void *rot, int precision, hipStream_t stream);

// Pair records over the half list; stats may be null.
void launch_pairs(const SysParams &p, const StatePtrs &s, const ListPtrs &l, const ForcePtrs &f, int precision,
                  unsigned long long *stats, hipStream_t stream);

// Per-particle sums of pair records in row order (fixed, atomic-free):
// F, tau, U_i, W_i; with kick != 0 also the closing velocity/angular
// momentum kick and (NVT) per-block kinetic partials.
void launch_gather(const SysParams &p, const StatePtrs &s, const OutPtrs &o, const ListPtrs &l, const ForcePtrs &f,
                   int precision, bool kick, double *ke_part, double *thermo, hipStream_t stream);

// Integrator pieces.  With NVT the gather's last workgroup applies the
// closing half step of the step and the opening half step of the next one;
// launch_nh_begin opens the first step of a call, launch_nh_end restores
// the state after the last closing half step and rescales the velocities.
void launch_nh_begin(const SysParams &p, const double *ke_part, int nblk, double *thermo, hipStream_t stream);
void launch_kick_drift(const SysParams &p, const StatePtrs &s, const OutPtrs &o, const ListPtrs &l,
                       const double *thermo, void *rot, int precision, hipStream_t stream);
void launch_kinetic(const SysParams &p, const StatePtrs &s, double *ke_part, hipStream_t stream);
void launch_nh_end(const SysParams &p, const StatePtrs &s, const double *ke_part, int nblk, double *thermo,
                   hipStream_t stream);
void launch_energy_partials(const SysParams &p, const StatePtrs &s, const OutPtrs &o, double *part,
                            hipStream_t stream);

constexpr int kBlock = 256;
inline int blocks_for(int n) { return (n + kBlock - 1) / kBlock; }
// The gather and the kinetic reduction map kGatherPer particles to each
// 256-thread block, which writes one kinetic partial.
constexpr int kGatherLanes = 4;
constexpr int kGatherPer = kBlock / kGatherLanes;
inline int gather_blocks(int n) { return (n + kGatherPer - 1) / kGatherPer; }

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

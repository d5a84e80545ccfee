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
enum Flag { FLAG_REBUILD = 0, FLAG_NBUILDS = 1, FLAG_MAXROW = 2, FLAG_NONFINITE = 3, FLAG_COUNT = 8 };
// Thermostat words (double): xi, eta, velocity scale, B-half-step pending.
enum Thermo { TH_XI = 0, TH_ETA = 1, TH_SCALE = 2, TH_PENDING = 3, TH_COUNT = 8 };
// Force work counters (unsigned long long).
enum Stat { ST_PAIRS = 0, ST_FEATURES = 1, ST_INCUT = 2, ST_LAUNCHES = 3, ST_NEAR = 4, ST_COUNT = 5 };

// Body-frame feature tables of one shape in precision T, laid out for LDS.
// Faces carry their outward unit normal n and offset o (n.x = o on the
// plane), the in-plane inward normal and offset of each loop edge (convex
// inside test), 2D face coordinates of each loop vertex (crossing-number
// test for concave faces) and 1/|edge|^2 for every segment projection.
template <typename T>
struct ShapeTab {
    int nv, ne, nf, pad0;
    T r, R, pad1, pad2;
    T v[DEM_MAX_VERTS][3];
    int e[DEM_MAX_EDGES][2];
    T ed[DEM_MAX_EDGES][3];      // edge vector b - a
    T einv[DEM_MAX_EDGES];       // 1 / |b - a|^2
    int foff[DEM_MAX_FACES + 1];
    int floop[DEM_MAX_LOOP];
    int fconvex[DEM_MAX_FACES];
    T fn[DEM_MAX_FACES][3];
    T fo[DEM_MAX_FACES];
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
};

// ---- launchers (all asynchronous on `stream`) ----
// Cell list + neighbour list; `gated` kernels exit at once unless the
// rebuild flag is set (so a captured step can contain them unconditionally).
void launch_build_lists(const SysParams &p, const StatePtrs &s, const ListPtrs &l, hipStream_t stream);

// Pair forces over the neighbour list; stats may be null.
void launch_forces(const SysParams &p, const StatePtrs &s, const OutPtrs &o, const ListPtrs &l, const void *tabs,
                   int precision, unsigned long long *stats, hipStream_t stream);

// Integrator pieces.
void launch_nh_begin(const SysParams &p, const double *ke_part, int nblk, double *thermo, hipStream_t stream);
void launch_kick_drift(const SysParams &p, const StatePtrs &s, const OutPtrs &o, const ListPtrs &l,
                       const double *thermo, hipStream_t stream);
void launch_kick(const SysParams &p, const StatePtrs &s, const OutPtrs &o, double *ke_part, double *thermo,
                 hipStream_t stream);
void launch_kinetic(const SysParams &p, const StatePtrs &s, double *ke_part, hipStream_t stream);
void launch_nh_end(const SysParams &p, const StatePtrs &s, const double *ke_part, int nblk, double *thermo,
                   hipStream_t stream);
void launch_energy_partials(const SysParams &p, const StatePtrs &s, const OutPtrs &o, double *part,
                            hipStream_t stream);

constexpr int kBlock = 256;
inline int blocks_for(int n) { return (n + kBlock - 1) / kBlock; }

}  // namespace dem

// Rigid-body integrator and reductions, FP64 (the closing kick is fused
// into the force gather, see dem_force.hip).
//
// Sec. IV.A: a second-order integrator; Sec. IV.C: a Nose-Hoover thermostat
// on translational and rotational degrees of freedom.  One step is
//   [NVT half step] kick (v, L by dt/2) - drift x by dt - free rotation -
//   forces - kick (dt/2) - [NVT half step],
// where the free rotation is the symmetric split about the body principal
// axes z(dt/2) y(dt/2) x(dt) y(dt/2) z(dt/2) (one rotation about z in 2D):
// a turn about body axis k by phi = h L_k / I_k right-multiplies q by the
// axis-angle quaternion and turns the body-frame L by -phi about that axis.
// The Nose-Hoover half step of length h on the single variable xi is
//   xi += h/2 (2K - g kT)/Q;  (v, L) *= exp(-xi h);  eta += xi h;
//   xi += h/2 (2K - g kT)/Q,
// with g = d N + d_rot N - d and Q = g kT tau_T^2.  The closing half step
// of a step and the opening half step of the next are computed together by
// k_replica_tail, one workgroup per replica after the force gather
// (dem_force.hip); their velocity factors are applied by the next
// kick-drift, and at the end
// of a call k_scale applies the closing factor alone, so a captured step
// needs no extra pass over the particles.
#include "dem_internal.h"

namespace dem {
namespace {

__device__ inline void quat_mul(double &w, double &x, double &y, double &z, double bw, double bx, double by,
                                double bz)
{
    double nw = w * bw - x * bx - y * by - z * bz;
    double nx = w * bx + x * bw + y * bz - z * by;
    double ny = w * by - x * bz + y * bw + z * bx;
    double nz = w * bz + x * by - y * bx + z * bw;
    w = nw;
    x = nx;
    y = ny;
    z = nz;
}

// sin and cos of an angle: for |a| <= 1/16 (every turn of a stable step)
// their Taylor series through the a^9 and a^10 terms in nested form, whose
// truncation is below 1e-19 relative there; sincos otherwise.
__device__ inline void sincos_turn(double a, double *sn, double *cs)
{
    if (fabs(a) <= 0.0625) {
        const double a2 = a * a;
        *sn = a * (1.0 - a2 * (1.0 / 6.0) * (1.0 - a2 * (1.0 / 20.0) * (1.0 - a2 * (1.0 / 42.0) * (1.0 - a2 * (1.0 / 72.0)))));
        *cs = 1.0 - a2 * 0.5 * (1.0 - a2 * (1.0 / 12.0) * (1.0 - a2 * (1.0 / 30.0) * (1.0 - a2 * (1.0 / 56.0) * (1.0 - a2 * (1.0 / 90.0)))));
    } else {
        sincos(a, sn, cs);
    }
}

// Free rotation about body axis k for time h.
__device__ inline void turn(double q[4], double L[3], const double I[3], int k, double h)
{
    if (I[k] <= 0.0) return;
    const double phi = h * L[k] / I[k];
    double sn, cs;
    sincos_turn(0.5 * phi, &sn, &cs);
    double b[3] = {0.0, 0.0, 0.0};
    b[k] = sn;
    quat_mul(q[0], q[1], q[2], q[3], cs, b[0], b[1], b[2]);
    const double s1 = 2.0 * sn * cs, c1 = (cs - sn) * (cs + sn);  // sin, cos of phi from the half angle
    const int a = (k + 1) % 3, c = (k + 2) % 3;
    const double La = L[a], Lc = L[c];
    L[a] = c1 * La + s1 * Lc;
    L[c] = -s1 * La + c1 * Lc;
}

// Body-frame torque R(q)^T tau.
__device__ inline void body_torque(const double q[4], double tx, double ty, double tz, double out[3])
{
    double R[9];
    quat_to_rot(q[0], q[1], q[2], q[3], R);
    out[0] = R[0] * tx + R[3] * ty + R[6] * tz;
    out[1] = R[1] * tx + R[4] * ty + R[7] * tz;
    out[2] = R[2] * tx + R[5] * ty + R[8] * tz;
}

__device__ inline double min_image(double d, double L) { return d - L * rint(d / L); }

template <int NT>
__device__ inline double block_sum(double v, double *sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
        if (t < off) sh[t] += sh[t + off];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Nose-Hoover half step on xi, eta; returns the velocity scale, updates K.
__device__ inline double nh_half(const SysParams &p, double &xi, double &eta, double &K)
{
    const double h = 0.5 * p.dt;
    xi += 0.5 * h * (2.0 * K - p.g * p.kT) / p.Qm;
    const double sc = exp(-xi * h);
    K *= sc * sc;
    eta += xi * h;
    xi += 0.5 * h * (2.0 * K - p.g * p.kT) / p.Qm;
    return sc;
}

// Replica of the wave's particles (chunks never straddle replicas), or -1.
__device__ inline int wave_replica(const BatchParams &b, const ListPtrs &l, int i)
{
    const int c = i / kChunk;
    return __builtin_amdgcn_readfirstlane(c < b.nchunk ? l.chunk_rep[c] : -1);
}

// Opening half step of a closed replica's next step, one workgroup per
// replica, from its kinetic partials (one per chunk, summed in order).
__global__ void __launch_bounds__(kBlock) k_nh_begin(BatchParams b, const SysParams *reps, const double *ke_part,
                                                        double *thermo, const int64_t *budget)
{
    __shared__ double sh[kBlock];
    const SysParams &p = reps[blockIdx.x];
    double *th = thermo + blockIdx.x * TH_COUNT;
    if (!p.live || p.n == 0 || (p.ensemble != DEM_NVT && p.ensemble != DEM_NPT) || budget[blockIdx.x] <= 0 ||
        th[TH_OPEN] != 0.0)
        return;
    const int c0 = p.off / kChunk, nc = (p.n + kChunk - 1) / kChunk;
    if (p.ensemble == DEM_NPT) {
        // thermostat half step, then barostat half step (from K_trans after
        // it, the virial of the current forces and the current box)
        double at = 0.0, ar = 0.0, aw = 0.0;
        for (int c = threadIdx.x; c < nc; c += blockDim.x) {
            at += ke_part[kKePer * (c0 + c)];
            ar += ke_part[kKePer * (c0 + c) + 1];
            aw += ke_part[kKePer * (c0 + c) + 2];
        }
        double Kt2 = 2.0 * block_sum<kBlock>(at, sh);
        const double Kr2 = 2.0 * block_sum<kBlock>(ar, sh);
        const double trW = block_sum<kBlock>(aw, sh);
        if (threadIdx.x != 0) return;
        double xi = th[TH_XI], eta = th[TH_ETA], veps = th[TH_VEPS];
        double K2 = Kt2 + Kr2;
        const double sa = nh_half_npt(p, xi, eta, K2, veps);
        Kt2 *= sa * sa;
        baro_half(p, Kt2, trW, veps);
        th[TH_XI] = xi;
        th[TH_ETA] = eta;
        th[TH_VEPS] = veps;
        th[TH_SB] = 1.0;
        th[TH_SA] = sa;
        th[TH_OPEN] = 1.0;
        npt_factors(p, veps, th);
        return;
    }
    double acc = 0.0;
    for (int c = threadIdx.x; c < nc; c += blockDim.x)
        acc += ke_part[kKePer * (c0 + c)] + ke_part[kKePer * (c0 + c) + 1];
    double K = block_sum<kBlock>(acc, sh);
    if (threadIdx.x != 0) return;
    double xi = th[TH_XI], eta = th[TH_ETA];
    const double sa = nh_half(p, xi, eta, K);
    th[TH_XI] = xi;
    th[TH_ETA] = eta;
    th[TH_SB] = 1.0;
    th[TH_SA] = sa;
    th[TH_OPEN] = 1.0;
}

// Start of a call: an NPT replica's box moves on to the box of its next
// step (TH_GROW times the box of the positions); end of a call: back to the
// box of the positions, which the tail of every step keeps in TH_BOXN.
__global__ void k_box_open(int nrep, SysParams *reps, ListPtrs l, const double *thermo, const int64_t *budget)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrep) return;
    SysParams &p = reps[r];
    const double *th = thermo + r * TH_COUNT;
    if (!p.live || p.ensemble != DEM_NPT || budget[r] <= 0) return;
    const double box[3] = {th[TH_BOXN] * th[TH_GROW], th[TH_BOXN + 1] * th[TH_GROW], th[TH_BOXN + 2] * th[TH_GROW]};
    set_box(p, box, l.flags + r * FLAG_COUNT);
}

__global__ void k_box_close(int nrep, SysParams *reps, ListPtrs l, const double *thermo)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrep) return;
    SysParams &p = reps[r];
    if (!p.live || p.ensemble != DEM_NPT) return;
    set_box(p, thermo + r * TH_COUNT + TH_BOXN, l.flags + r * FLAG_COUNT);
}

// End of a call: the velocities take the pending closing factor.
__global__ void k_scale(BatchParams b, const SysParams *reps, StatePtrs s, ListPtrs l, const double *thermo)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = wave_replica(b, l, i);
    if (r < 0 || i >= reps[r].off + reps[r].n) return;
    const double sc = thermo[r * TH_COUNT + TH_SB];
    if ((reps[r].ensemble != DEM_NVT && reps[r].ensemble != DEM_NPT) || sc == 1.0) return;
    s.vx[i] *= sc;
    s.vy[i] *= sc;
    s.vz[i] *= sc;
    s.Lx[i] *= sc;
    s.Ly[i] *= sc;
    s.Lz[i] *= sc;
}

__global__ void k_nh_close(int nrep, double *thermo)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nrep) thermo[r * TH_COUNT + TH_SB] = 1.0;
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kChunk) k_kick_drift(BatchParams b, const SysParams *reps, StatePtrs s, OutPtrs o,
                                                          ListPtrs l, const double *thermo, const int64_t *budget,
                                                          void *rot, PartRec64 *rec64)
{
    const int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i == 0) l.gflags[G_STAMP] += 1;  // this step's force evaluation
    // the particle's own values are requested with the replica's parameters
    // instead of after them (within the length of the state arrays)
    double q[4] = {1.0, 0.0, 0.0, 0.0}, v0[3] = {0.0, 0.0, 0.0}, L0[3] = {0.0, 0.0, 0.0};
    double F0[3] = {0.0, 0.0, 0.0}, T0[3] = {0.0, 0.0, 0.0}, x[3] = {0.0, 0.0, 0.0};
    int img[3] = {0, 0, 0}, sid = 0;
    if (i < b.nstate) {
        sid = s.sid[i];
        x[0] = s.x[i];
        x[1] = s.y[i];
        v0[0] = s.vx[i];
        v0[1] = s.vy[i];
        L0[2] = s.Lz[i];
        F0[0] = o.Fx[i];
        F0[1] = o.Fy[i];
        T0[2] = o.Tz[i];
        if (DIM == 3) {
            x[2] = s.z[i];
            v0[2] = s.vz[i];
            L0[0] = s.Lx[i];
            L0[1] = s.Ly[i];
            F0[2] = o.Fz[i];
            T0[0] = o.Tx[i];
            T0[1] = o.Ty[i];
        }
        q[0] = s.qw[i];
        q[1] = s.qx[i];
        q[2] = s.qy[i];
        q[3] = s.qz[i];
        img[0] = s.image[3 * i];
        img[1] = s.image[3 * i + 1];
        img[2] = s.image[3 * i + 2];
    }
    double xl[3] = {0.0, 0.0, 0.0};  // position at the last list build (the library's N slots)
    if (i < b.N)
        for (int a = 0; a < DIM; ++a) xl[a] = l.xlast[(size_t)a * b.N + i];
    const int r = wave_replica(b, l, i);
    if (r < 0) return;
    // the replica's per-step values are requested together with its
    // parameters, not one round trip after another (this kernel writes
    // none of them; the thermostat slots exist for every replica)
    const int64_t left = budget[r];
    const double *thr = thermo + r * TH_COUNT;
    const double th_sb = thr[TH_SB], th_sa = thr[TH_SA];
    const int32_t rebuild = l.flags[r * FLAG_COUNT + FLAG_REBUILD];
    const SysParams &p = reps[r];
    if (i >= p.off + p.n || left <= 0) return;
    // pending thermostat factors: the closing half step of the last step,
    // then the opening half step of this one (1 and 1 without a thermostat)
    const bool npt = p.ensemble == DEM_NPT;
    const bool nvt = p.ensemble == DEM_NVT || npt;
    const double sb = nvt ? th_sb : 1.0;
    const double sa = nvt ? th_sa : 1.0;
    const double hm = 0.5 * p.dt / p.mass[sid];
    const double I[3] = {p.inertia[sid][0], p.inertia[sid][1], p.inertia[sid][2]};
    double v[3] = {(v0[0] * sb) * sa + hm * F0[0], (v0[1] * sb) * sa + hm * F0[1], 0.0};
    double grow = 1.0, vfac = p.dt;
    if (npt) {
        // the exact flow of the kick with the barostat's friction, and of
        // the drift with the box growing by `grow` this step
        const double damp = thr[TH_DAMP], fk = thr[TH_FK] / p.mass[sid];
        grow = thr[TH_GROW];
        vfac = thr[TH_VFAC];
        for (int a = 0; a < 3; ++a) v[a] = ((v0[a] * sb) * sa) * damp + fk * F0[a];
        if (DIM == 2) v[2] = 0.0;
    }
    double L[3];
    if (DIM == 3) {
        if (!npt) v[2] = (v0[2] * sb) * sa + hm * F0[2];
        double tb[3];
        body_torque(q, T0[0], T0[1], T0[2], tb);
        L[0] = (L0[0] * sb) * sa + 0.5 * p.dt * tb[0];
        L[1] = (L0[1] * sb) * sa + 0.5 * p.dt * tb[1];
        L[2] = (L0[2] * sb) * sa + 0.5 * p.dt * tb[2];
    } else {
        L[0] = 0.0;
        L[1] = 0.0;
        L[2] = (L0[2] * sb) * sa + 0.5 * p.dt * T0[2];
    }
    for (int a = 0; a < DIM; ++a) {
        double xa = npt ? x[a] * grow + vfac * v[a] : x[a] + p.dt * v[a];
        if (xa >= p.box[a]) {
            xa -= p.box[a];
            img[a] += 1;
        } else if (xa < 0.0) {
            xa += p.box[a];
            img[a] -= 1;
        }
        x[a] = xa;
    }
    if (DIM == 3) {
        turn(q, L, I, 2, 0.5 * p.dt);
        turn(q, L, I, 1, 0.5 * p.dt);
        turn(q, L, I, 0, p.dt);
        turn(q, L, I, 1, 0.5 * p.dt);
        turn(q, L, I, 2, 0.5 * p.dt);
    } else {
        turn(q, L, I, 2, p.dt);
    }
    const double qn = 1.0 / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int a = 0; a < 4; ++a) q[a] *= qn;
    s.qw[i] = q[0];
    s.qx[i] = q[1];
    s.qy[i] = q[2];
    s.qz[i] = q[3];
    {  // the force pass's record: new position, rotation of the new orientation, shape
        double R[9];
        quat_to_rot(q[0], q[1], q[2], q[3], R);
        PartRec<T> rc;
        rc.x = x[0];
        rc.y = x[1];
        rc.z = x[2];
        for (int k = 0; k < 9; ++k) rc.R[k] = (T)R[k];
        rc.sid = sid;
        reinterpret_cast<PartRec<T> *>(rot)[i] = rc;
        if (sizeof(T) == 4) rec64[i] = PartRec64{x[0], x[1], x[2], q[0], q[1], q[2], q[3], 0.0};
    }
    s.x[i] = x[0];
    s.y[i] = x[1];
    s.vx[i] = v[0];
    s.vy[i] = v[1];
    if (DIM == 3) {
        s.z[i] = x[2];
        s.vz[i] = v[2];
        s.Lx[i] = L[0];
        s.Ly[i] = L[1];
    }
    s.Lz[i] = L[2];
    s.image[3 * i] = img[0];
    s.image[3 * i + 1] = img[1];
    s.image[3 * i + 2] = img[2];
    if (rebuild != 0) {
        // this step rebuilds the lists from the positions after this drift:
        // the particle goes into its cell now (and the new pair total
        // restarts for the row workgroups to add to); this step's forces
        // still use the lists in place, which the trigger of the previous
        // step has kept valid for these positions
        if (i == p.off) l.flags[r * FLAG_COUNT + FLAG_NEWPAIRS] = 0;
        cell_insert(p, l, i, x[0], x[1], x[2]);
    } else {
        // The next step rebuilds them if the displacement since the last
        // build, plus one more step like this one, exceeds rebuild_frac * skin
        // (so no force is evaluated on a list older than that).
        double d2 = 0.0, v2 = 0.0;
        if (npt) {
            // under the barostat the lists were built in the box
            // box_build: a particle's displacement is taken from its build
            // position carried along with the box, and a shrinking box brings
            // pairs beyond r_list closer by (1 - s) r_list (s = the box's
            // scale since the build, one more step included)
            const double lam = p.box[0] / p.box_build[0];
            for (int a = 0; a < DIM; ++a) {
                const double d = min_image(x[a] - lam * xl[a], p.box[a]);
                d2 += d * d;
                v2 += v[a] * v[a];
            }
            const double shrink = fmax(0.0, 1.0 - lam * grow) * 0.5 * sqrt(p.rl2);
            const double reach = sqrt(d2) + p.dt * sqrt(v2) + shrink;
            if (reach * reach > p.disp2) atomicOr(&l.flags[r * FLAG_COUNT + FLAG_TRIGGER], 1);
        } else {
        for (int a = 0; a < DIM; ++a) {
            const double d = min_image(x[a] - xl[a], p.box[a]);
            d2 += d * d;
            v2 += v[a] * v[a];
        }
        const double reach = sqrt(d2) + p.dt * sqrt(v2);
        if (reach * reach > p.disp2) atomicOr(&l.flags[r * FLAG_COUNT + FLAG_TRIGGER], 1);
        }
    }
    if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]) && isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2])))
        atomicOr(&l.flags[r * FLAG_COUNT + FLAG_NONFINITE], 1);
}

// Per-chunk kinetic partials of the current state, with the particle-to-
// block mapping of the gather (one chunk per block).
__global__ void __launch_bounds__(kGatherBlock) k_kinetic(BatchParams b, const SysParams *reps, StatePtrs s, OutPtrs o,
                                                       ListPtrs l, double *ke_part)
{
    __shared__ double sh[kGatherBlock];
    const int r = l.chunk_rep[blockIdx.x];
    if (r < 0) return;
    const SysParams &p = reps[r];
    const int i = blockIdx.x * kGatherPer + threadIdx.x / kGatherLanes;
    double kt = 0.0, kr = 0.0, tw = 0.0;
    if (i < p.off + p.n && (threadIdx.x % kGatherLanes) == 0) {
        const int sid = s.sid[i];
        const double m = p.mass[sid];
        kt = 0.5 * m * (s.vx[i] * s.vx[i] + s.vy[i] * s.vy[i] + s.vz[i] * s.vz[i]);
        const double L[3] = {s.Lx[i], s.Ly[i], s.Lz[i]};
        for (int a = 0; a < 3; ++a)
            if (p.inertia[sid][a] > 0.0) kr += 0.5 * L[a] * L[a] / p.inertia[sid][a];
        if (p.ensemble == DEM_NPT)
            tw = o.W[i] + o.W[(size_t)4 * b.wstride + i] + (p.dim == 3 ? o.W[(size_t)8 * b.wstride + i] : 0.0);
    }
    kt = block_sum<kGatherBlock>(kt, sh);
    kr = block_sum<kGatherBlock>(kr, sh);
    tw = block_sum<kGatherBlock>(tw, sh);
    if (threadIdx.x == 0) {
        ke_part[kKePer * blockIdx.x] = kt;
        ke_part[kKePer * blockIdx.x + 1] = kr;
        ke_part[kKePer * blockIdx.x + 2] = tw;
    }
}

// Per-chunk partials of U, K_trans, K_rot and W (9) of chunks c0, c0 + 1,
// ...: part[(chunk - c0) * 12 + c].
__global__ void __launch_bounds__(kChunk) k_energy_partials(BatchParams b, const SysParams *reps, StatePtrs s,
                                                               OutPtrs o, ListPtrs l, double *part, int c0)
{
    __shared__ double sh[kChunk];
    const int ch = c0 + (int)blockIdx.x;
    const int r = l.chunk_rep[ch];
    if (r < 0) return;
    const SysParams &p = reps[r];
    const int i = ch * kChunk + threadIdx.x;
    double val[12];
    for (int c = 0; c < 12; ++c) val[c] = 0.0;
    if (i < p.off + p.n) {
        const int sid = s.sid[i];
        val[0] = o.U[i];
        val[1] = 0.5 * p.mass[sid] * (s.vx[i] * s.vx[i] + s.vy[i] * s.vy[i] + s.vz[i] * s.vz[i]);
        const double L[3] = {s.Lx[i], s.Ly[i], s.Lz[i]};
        for (int a = 0; a < 3; ++a)
            if (p.inertia[sid][a] > 0.0) val[2] += 0.5 * L[a] * L[a] / p.inertia[sid][a];
        for (int c = 0; c < 9; ++c) val[3 + c] = o.W[(size_t)c * b.wstride + i];
    }
    for (int c = 0; c < 12; ++c) {
        const double v = block_sum<kChunk>(val[c], sh);
        if (threadIdx.x == 0) part[12 * blockIdx.x + c] = v;
    }
}

}  // namespace

void launch_nh_begin(const Launch &L, hipStream_t stream)
{
    if (L.b.nrep == 0) return;
    k_nh_begin<<<L.b.nrep, kBlock, 0, stream>>>(L.b, L.reps, L.ke_part, L.thermo, L.budget);
    k_box_open<<<blocks_for(L.b.nrep), kBlock, 0, stream>>>(L.b.nrep, const_cast<SysParams *>(L.reps), L.l, L.thermo,
                                                          L.budget);
}

void launch_nh_end(const Launch &L, hipStream_t stream)
{
    if (L.b.nrep == 0) return;
    const int nr = (L.b.nrep + kBlock - 1) / kBlock;
    if (L.b.nchunk > 0) k_scale<<<blocks_for(L.b.nchunk * kChunk), kBlock, 0, stream>>>(L.b, L.reps, L.s, L.l, L.thermo);
    k_nh_close<<<nr, kBlock, 0, stream>>>(L.b.nrep, L.thermo);
    k_box_close<<<nr, kBlock, 0, stream>>>(L.b.nrep, const_cast<SysParams *>(L.reps), L.l, L.thermo);
}

template <typename T>
void kick_drift_t(const Launch &L, hipStream_t stream)
{
    // one wavefront (one chunk) per block: the chunks spread over as many
    // CUs as there are chunks
    const int nb = pad8(L.b.nchunk);
    if (L.b.dim == 3)
        k_kick_drift<T, 3><<<nb, kChunk, 0, stream>>>(L.b, L.reps, L.s, L.o, L.l, L.thermo, L.budget, L.f.rot,
                                                       L.f.rec64);
    else
        k_kick_drift<T, 2><<<nb, kChunk, 0, stream>>>(L.b, L.reps, L.s, L.o, L.l, L.thermo, L.budget, L.f.rot,
                                                       L.f.rec64);
}

void launch_kick_drift(const Launch &L, hipStream_t stream)
{
    if (L.b.nchunk == 0) return;
    if (L.precision == DEM_FP32) kick_drift_t<float>(L, stream);
    else kick_drift_t<double>(L, stream);
}

void launch_kinetic(const Launch &L, hipStream_t stream)
{
    if (L.b.nchunk == 0) return;
    k_kinetic<<<L.b.nchunk, kGatherBlock, 0, stream>>>(L.b, L.reps, L.s, L.o, L.l, L.ke_part);
}

void launch_energy_partials(const Launch &L, double *part, hipStream_t stream)
{
    if (L.b.nchunk == 0) return;
    k_energy_partials<<<L.b.nchunk, kChunk, 0, stream>>>(L.b, L.reps, L.s, L.o, L.l, part, 0);
}

// The partials of chunks c0 .. c0 + nchunks - 1 into part[0 .. 12 nchunks),
// then their totals in chunk order (the order of the host sum of
// dem_replica_energy, so the bits agree) into total[0 .. 12).
__global__ void k_sum_partials(const double *part, int nchunks, double *total)
{
    const int c = threadIdx.x;
    if (c >= 12) return;
    double acc = 0.0;
    for (int k = 0; k < nchunks; ++k) acc += part[(size_t)12 * k + c];
    total[c] = acc;
}

void launch_energy_totals(const Launch &L, int c0, int nchunks, double *part, double *total, hipStream_t stream)
{
    if (nchunks > 0) k_energy_partials<<<nchunks, kChunk, 0, stream>>>(L.b, L.reps, L.s, L.o, L.l, part, c0);
    k_sum_partials<<<1, 64, 0, stream>>>(part, nchunks, total);
}

}  // namespace dem

// Pair force, torque, energy and virial of rounded polytopes.
//
// Sec. II, Eq. 1 (3D): U_ij sums the WCA potential over every edge-edge
// pair, every (vertex of i, face of j) pair and every (vertex of j, face of
// i) pair; Eq. 2 (2D): over every (vertex of i, edge of j) and (vertex of j,
// edge of i) pair; each at the nearest points of the two features.  The
// potential is WCA (Eq. 3-4) with sigma_ij = r_i + r_j; the force acts along
// the nearest-point line and the torque on each particle comes from its own
// interaction point.  Nearly parallel edges interact at the midpoints of
// their overlap (Sec. II, paragraph on parallel edges).
//
// Mapping to gfx950: one wave64 per particle i over a full neighbour list,
// so every particle sums its own force with no atomics and a fixed order.
// For each neighbour j inside R_i + R_j + r_cut the whole wave shares the
// pair transform (j's frame relative to i's, built in FP64 and rounded
// once), and the 64 lanes stride over the feature-pair problems.  All
// geometry is done in i's body frame (vertex-face problems in the face
// owner's frame) against shape tables staged in LDS.  Per-lane partial sums
// are reduced across the wave in FP64 with cross-lane shuffles.
#include "dem_internal.h"

namespace dem {
namespace {

template <typename T>
struct V3 {
    T x, y, z;
};
template <typename T>
__device__ inline V3<T> v3(T a, T b, T c) { return {a, b, c}; }
template <typename T>
__device__ inline V3<T> operator+(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename T>
__device__ inline V3<T> operator-(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T>
__device__ inline V3<T> operator*(T s, V3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <typename T>
__device__ inline T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T>
__device__ inline V3<T> cross(V3<T> a, V3<T> b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename T>
__device__ inline V3<T> ld3(const T (&a)[3]) { return {a[0], a[1], a[2]}; }
template <typename T>
__device__ inline T clamp01(T t) { return t < T(0) ? T(0) : (t > T(1) ? T(1) : t); }

// Rotation (3x3, row-major) as rows; apply and apply-transpose.
template <typename T>
struct M3 {
    T m[9];
};
template <typename T>
__device__ inline V3<T> mul(const M3<T> &R, V3<T> v)
{
    return {R.m[0] * v.x + R.m[1] * v.y + R.m[2] * v.z, R.m[3] * v.x + R.m[4] * v.y + R.m[5] * v.z,
            R.m[6] * v.x + R.m[7] * v.y + R.m[8] * v.z};
}
template <typename T>
__device__ inline V3<T> mulT(const M3<T> &R, V3<T> v)
{
    return {R.m[0] * v.x + R.m[3] * v.y + R.m[6] * v.z, R.m[1] * v.x + R.m[4] * v.y + R.m[7] * v.z,
            R.m[2] * v.x + R.m[5] * v.y + R.m[8] * v.z};
}

__device__ inline M3<double> quat_rot(double w, double x, double y, double z)
{
    M3<double> R;
    R.m[0] = 1.0 - 2.0 * (y * y + z * z);
    R.m[1] = 2.0 * (x * y - w * z);
    R.m[2] = 2.0 * (x * z + w * y);
    R.m[3] = 2.0 * (x * y + w * z);
    R.m[4] = 1.0 - 2.0 * (x * x + z * z);
    R.m[5] = 2.0 * (y * z - w * x);
    R.m[6] = 2.0 * (x * z - w * y);
    R.m[7] = 2.0 * (y * z + w * x);
    R.m[8] = 1.0 - 2.0 * (x * x + y * y);
    return R;
}

// Nearest point of the closed segment a + t u (t in [0,1]) to p.
template <typename T>
__device__ inline V3<T> seg_point(V3<T> p, V3<T> a, V3<T> u, T inv_uu)
{
    return a + clamp01(dot(p - a, u) * inv_uu) * u;
}

// Nearest point of face f of shape S to p, both in S's body frame.  Returns
// false when the plane distance alone already reaches the cutoff (the
// polygon distance is at least the plane distance).  Inside test: in-plane
// half-spaces for convex faces, crossing number for concave ones; outside,
// the nearest point lies on the face's own boundary edges.
template <typename T>
__device__ inline bool face_point(const ShapeTab<T> &S, int f, V3<T> p, T rc, V3<T> &q)
{
    V3<T> n = ld3(S.fn[f]);
    T sd = dot(n, p) - S.fo[f];
    if (fabs(sd) >= rc) return false;
    const int k0 = S.foff[f], k1 = S.foff[f + 1];
    bool inside;
    if (S.fconvex[f]) {
        inside = true;
        for (int k = k0; k < k1; ++k)
            inside = inside && (dot(ld3(S.lnrm[k]), p) >= S.loff[k]);
    } else {
        V3<T> e1 = ld3(S.fe1[f]);
        V3<T> e2 = cross(n, e1);
        V3<T> o = ld3(S.v[S.floop[k0]]);
        T px = dot(p - o, e1), py = dot(p - o, e2);
        inside = false;
        for (int k = k0; k < k1; ++k) {
            int kn = (k + 1 < k1) ? k + 1 : k0;
            T ax = S.lxy[k][0], ay = S.lxy[k][1], bx = S.lxy[kn][0], by = S.lxy[kn][1];
            if ((ay > py) != (by > py)) {
                T xc = ax + (py - ay) * (bx - ax) / (by - ay);
                if (px < xc) inside = !inside;
            }
        }
    }
    if (inside) {
        q = p - sd * n;
        return true;
    }
    T best = T(3.0e38);
    for (int k = k0; k < k1; ++k) {
        int kn = (k + 1 < k1) ? k + 1 : k0;
        V3<T> a = ld3(S.v[S.floop[k]]);
        V3<T> c = seg_point(p, a, ld3(S.v[S.floop[kn]]) - a, S.linv[k]);
        V3<T> d = p - c;
        T d2 = dot(d, d);
        if (d2 < best) {
            best = d2;
            q = c;
        }
    }
    return true;
}

// Closest points of segments p1 + s d1 and p2 + t d2 (s, t in [0,1]).
// Non-parallel: the clamped line solution (Ericson, Real-Time Collision
// Detection, 2005, Sec. 5.1.9) with the cross-product form of its
// denominator.  Nearly parallel: each point is the midpoint of its segment's
// overlap with the other segment's projection, or the facing endpoint.
template <typename T>
__device__ inline void seg_seg(V3<T> p1, V3<T> d1, T a, V3<T> p2, V3<T> d2, T e, T par_s2, V3<T> &P, V3<T> &Q)
{
    V3<T> r = p1 - p2;
    T b = dot(d1, d2), c = dot(d1, r), f = dot(d2, r);
    V3<T> cr = cross(d1, d2);
    T den = dot(cr, cr);
    T s, t;
    if (den < par_s2 * a * e) {
        T ia = T(1) / a, ie = T(1) / e;
        T t0 = -c * ia, t1 = (b - c) * ia;
        T lo = fmax(T(0), fmin(t0, t1)), hi = fmin(T(1), fmax(t0, t1));
        s = (lo <= hi) ? T(0.5) * (lo + hi) : (fmax(t0, t1) < T(0) ? T(0) : T(1));
        T u0 = f * ie, u1 = (f + b) * ie;
        lo = fmax(T(0), fmin(u0, u1));
        hi = fmin(T(1), fmax(u0, u1));
        t = (lo <= hi) ? T(0.5) * (lo + hi) : (fmax(u0, u1) < T(0) ? T(0) : T(1));
    } else {
        s = clamp01((b * f - c * e) / den);
        t = (b * s + f) / e;
        if (t < T(0)) {
            t = T(0);
            s = clamp01(-c / a);
        } else if (t > T(1)) {
            t = T(1);
            s = clamp01((b - c) / a);
        }
    }
    P = p1 + s * d1;
    Q = p2 + t * d2;
}

template <typename T>
struct Acc {
    V3<T> F, Tq;
    T U;
    T M[9];  // sum over pairs of d_ij (x) f (d in space frame, f in i's frame)
};

// WCA (Eq. 3-4): adds the contribution of interaction points P (on i) and
// Q (on j), both in i's frame, if |P - Q| < r_cut.
template <typename T>
__device__ inline int add_wca(Acc<T> &A, V3<T> P, V3<T> Q, V3<T> dsp, T sig2, T rc2, T eps)
{
    V3<T> rho = P - Q;
    T r2 = dot(rho, rho);
    if (!(r2 < rc2)) return 0;
    T ir2 = T(1) / r2;
    T s2 = sig2 * ir2;
    T s6 = s2 * s2 * s2;
    T u = T(4) * eps * s6 * (s6 - T(1)) + eps;
    T fr = T(24) * eps * s6 * (T(2) * s6 - T(1)) * ir2;
    V3<T> f = fr * rho;
    A.F = A.F + f;
    A.Tq = A.Tq + cross(P, f);
    A.U += u;
    A.M[0] += dsp.x * f.x; A.M[1] += dsp.x * f.y; A.M[2] += dsp.x * f.z;
    A.M[3] += dsp.y * f.x; A.M[4] += dsp.y * f.y; A.M[5] += dsp.y * f.z;
    A.M[6] += dsp.z * f.x; A.M[7] += dsp.z * f.y; A.M[8] += dsp.z * f.z;
    return 1;
}

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double min_image(double d, double L) { return d - L * rint(d / L); }

constexpr int kWaves = 4;  // waves (particles) per block

template <typename T, int DIM>
__global__ void __launch_bounds__(64 * kWaves) k_forces(SysParams p, StatePtrs s, OutPtrs o, ListPtrs l,
                                                           const ShapeTab<T> *__restrict__ gtab,
                                                           unsigned long long *stats)
{
    extern __shared__ __align__(16) unsigned char smem[];
    ShapeTab<T> *tab = reinterpret_cast<ShapeTab<T> *>(smem);
    {
        const int words = p.n_shapes * (int)(sizeof(ShapeTab<T>) / 4);
        const uint32_t *src = reinterpret_cast<const uint32_t *>(gtab);
        uint32_t *dst = reinterpret_cast<uint32_t *>(smem);
        for (int w = threadIdx.x; w < words; w += blockDim.x) dst[w] = src[w];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && l.flags[FLAG_REBUILD] != 0) {
        // the lists consumed by this launch are fresh: count the build and clear the trigger
        l.flags[FLAG_REBUILD] = 0;
        l.flags[FLAG_NBUILDS] += 1;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (i >= p.n) return;
    const int n = p.n;

    const double xi = s.x[i], yi = s.y[i], zi = (DIM == 3) ? s.z[i] : 0.0;
    const M3<double> Ri = quat_rot(s.qw[i], s.qx[i], s.qy[i], s.qz[i]);
    const int si = s.sid[i];
    const ShapeTab<T> &Si = tab[si];

    Acc<T> A;
    A.F = v3<T>(0, 0, 0);
    A.Tq = v3<T>(0, 0, 0);
    A.U = 0;
    for (int k = 0; k < 9; ++k) A.M[k] = 0;
    unsigned long long c_pairs = 0, c_feat = 0, c_in = 0, c_near = 0;

    const int nn = l.n_nbr[i];
    for (int k = 0; k < nn; ++k) {
        const int j = l.nbr[(size_t)k * n + i];
        const double dx = min_image(s.x[j] - xi, p.box[0]);
        const double dy = min_image(s.y[j] - yi, p.box[1]);
        const double dz = (DIM == 3) ? min_image(s.z[j] - zi, p.box[2]) : 0.0;
        const int sj = s.sid[j];
        const double bound = p.R[si] + p.R[sj] + kWcaCut * (p.rad[si] + p.rad[sj]);
        if (dx * dx + dy * dy + dz * dz >= bound * bound) continue;
        const ShapeTab<T> &Sj = tab[sj];

        // j's frame relative to i's frame, in FP64, rounded once to T
        const M3<double> Rj = quat_rot(s.qw[j], s.qx[j], s.qy[j], s.qz[j]);
        M3<T> Rr;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                Rr.m[3 * a + b] = (T)(Ri.m[a] * Rj.m[b] + Ri.m[3 + a] * Rj.m[3 + b] + Ri.m[6 + a] * Rj.m[6 + b]);
        const V3<T> t = v3<T>((T)(Ri.m[0] * dx + Ri.m[3] * dy + Ri.m[6] * dz),
                              (T)(Ri.m[1] * dx + Ri.m[4] * dy + Ri.m[7] * dz),
                              (T)(Ri.m[2] * dx + Ri.m[5] * dy + Ri.m[8] * dz));
        const V3<T> dsp = v3<T>((T)dx, (T)dy, (T)dz);
        const double sigd = p.rad[si] + p.rad[sj];
        const T sig2 = (T)(sigd * sigd);
        const T rc = (T)(kWcaCut * sigd);
        const T rc2 = rc * rc;
        const T eps = (T)p.eps;

        int nA, nB, nC;
        if (DIM == 3) {
            nA = Si.nv * Sj.nf;
            nB = Sj.nv * Si.nf;
            nC = Si.ne * Sj.ne;
        } else {
            nA = Si.nv * Sj.ne;
            nB = Sj.nv * Si.ne;
            nC = 0;
        }
        const int total = nA + nB + nC;
        c_pairs += 1;
        c_feat += total;
        for (int q = lane; q < total; q += 64) {
            V3<T> P, Q;
            bool ok = true;
            if (q < nA) {
                if (DIM == 3) {
                    // vertex a of i against face f of j, in j's frame
                    const int a = q / Sj.nf, f = q - a * Sj.nf;
                    const V3<T> va = ld3(Si.v[a]);
                    V3<T> qj;
                    ok = face_point(Sj, f, mulT(Rr, va - t), rc, qj);
                    P = va;
                    Q = t + mul(Rr, qj);
                } else {
                    // vertex a of i against edge e of j, in j's frame
                    const int a = q / Sj.ne, e = q - a * Sj.ne;
                    const V3<T> va = ld3(Si.v[a]);
                    const V3<T> qj = seg_point(mulT(Rr, va - t), ld3(Sj.v[Sj.e[e][0]]), ld3(Sj.ed[e]), Sj.einv[e]);
                    P = va;
                    Q = t + mul(Rr, qj);
                }
            } else if (q < nA + nB) {
                const int qq = q - nA;
                if (DIM == 3) {
                    // vertex b of j against face f of i, in i's frame
                    const int b = qq / Si.nf, f = qq - b * Si.nf;
                    const V3<T> vb = t + mul(Rr, ld3(Sj.v[b]));
                    ok = face_point(Si, f, vb, rc, P);
                    Q = vb;
                } else {
                    const int b = qq / Si.ne, e = qq - b * Si.ne;
                    const V3<T> vb = t + mul(Rr, ld3(Sj.v[b]));
                    P = seg_point(vb, ld3(Si.v[Si.e[e][0]]), ld3(Si.ed[e]), Si.einv[e]);
                    Q = vb;
                }
            } else {
                // edge ei of i against edge ej of j, in i's frame
                const int qq = q - nA - nB;
                const int ei = qq / Sj.ne, ej = qq - ei * Sj.ne;
                const V3<T> a0 = ld3(Si.v[Si.e[ei][0]]);
                const V3<T> b0 = t + mul(Rr, ld3(Sj.v[Sj.e[ej][0]]));
                const V3<T> d2 = mul(Rr, ld3(Sj.ed[ej]));
                seg_seg(a0, ld3(Si.ed[ei]), T(1) / Si.einv[ei], b0, d2, T(1) / Sj.einv[ej], (T)p.par_s2, P, Q);
            }
            if (DIM == 3 && q < nA + nB) c_near += ok ? 1 : 0;
            if (ok) c_in += add_wca(A, P, Q, dsp, sig2, rc2, eps);
        }
    }

    // wave reduction in FP64
    double F[3] = {wave_sum((double)A.F.x), wave_sum((double)A.F.y), wave_sum((double)A.F.z)};
    double Tq[3] = {wave_sum((double)A.Tq.x), wave_sum((double)A.Tq.y), wave_sum((double)A.Tq.z)};
    double U = wave_sum((double)A.U);
    double M[9];
    for (int k = 0; k < 9; ++k) M[k] = wave_sum((double)A.M[k]);
    if (stats) {
        unsigned long long in_w = c_in, near_w = c_near;
        for (int off = 32; off > 0; off >>= 1) {
            in_w += __shfl_xor(in_w, off, 64);
            near_w += __shfl_xor(near_w, off, 64);
        }
        if (lane == 0) {
            atomicAdd(&stats[ST_PAIRS], c_pairs);
            atomicAdd(&stats[ST_FEATURES], c_feat);
            atomicAdd(&stats[ST_INCUT], in_w);
            atomicAdd(&stats[ST_NEAR], near_w);
            if (i == 0) atomicAdd(&stats[ST_LAUNCHES], 1ull);
        }
    }
    if (lane == 0) {
        // back to the space frame: F = R_i f, tau = R_i (P x f), W_i = -1/2 M R_i^T
        o.Fx[i] = Ri.m[0] * F[0] + Ri.m[1] * F[1] + Ri.m[2] * F[2];
        o.Fy[i] = Ri.m[3] * F[0] + Ri.m[4] * F[1] + Ri.m[5] * F[2];
        o.Fz[i] = (DIM == 3) ? Ri.m[6] * F[0] + Ri.m[7] * F[1] + Ri.m[8] * F[2] : 0.0;
        if (DIM == 3) {
            o.Tx[i] = Ri.m[0] * Tq[0] + Ri.m[1] * Tq[1] + Ri.m[2] * Tq[2];
            o.Ty[i] = Ri.m[3] * Tq[0] + Ri.m[4] * Tq[1] + Ri.m[5] * Tq[2];
        } else {
            o.Tx[i] = 0.0;
            o.Ty[i] = 0.0;
        }
        o.Tz[i] = Ri.m[6] * Tq[0] + Ri.m[7] * Tq[1] + Ri.m[8] * Tq[2];
        o.U[i] = 0.5 * U;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                o.W[(size_t)(3 * a + b) * n + i] =
                    -0.5 * (M[3 * a] * Ri.m[3 * b] + M[3 * a + 1] * Ri.m[3 * b + 1] + M[3 * a + 2] * Ri.m[3 * b + 2]);
    }
}

}  // namespace

void launch_forces(const SysParams &p, const StatePtrs &s, const OutPtrs &o, const ListPtrs &l, const void *tabs,
                   int precision, unsigned long long *stats, hipStream_t stream)
{
    if (p.n == 0) return;
    const int grid = (p.n + kWaves - 1) / kWaves;
    const int block = 64 * kWaves;
    if (precision == DEM_FP32) {
        const size_t sh = (size_t)p.n_shapes * sizeof(ShapeTab<float>);
        auto *t = reinterpret_cast<const ShapeTab<float> *>(tabs);
        if (p.dim == 3)
            k_forces<float, 3><<<grid, block, sh, stream>>>(p, s, o, l, t, stats);
        else
            k_forces<float, 2><<<grid, block, sh, stream>>>(p, s, o, l, t, stats);
    } else {
        const size_t sh = (size_t)p.n_shapes * sizeof(ShapeTab<double>);
        auto *t = reinterpret_cast<const ShapeTab<double> *>(tabs);
        if (p.dim == 3)
            k_forces<double, 3><<<grid, block, sh, stream>>>(p, s, o, l, t, stats);
        else
            k_forces<double, 2><<<grid, block, sh, stream>>>(p, s, o, l, t, stats);
    }
}

}  // namespace dem

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
// Mapping to gfx950 (two kernels):
//  1. k_pairs: one wave64 per unordered pair of the half list (grid-stride).
//     The wave builds j's frame relative to i's once, transforms both
//     vertex sets across (one lane per vertex, kept in LDS), then runs the
//     contact search: every feature pair of Eq. 1/2 gets a cheap
//     conservative test (plane distance and bounding circle for
//     vertex-face, bounding spheres for edge-edge and vertex-edge), and the
//     survivors are compacted into a per-wave LDS queue with ballot/popcount
//     so the exact nearest-point and WCA work runs on dense lanes.  The wave
//     reduces force and both torques in FP64 and writes one record per pair.
//  2. k_gather: one thread per particle sums its row of pair records in row
//     order (no atomics, deterministic) into F, tau, U_i and W_i, optionally
//     fused with the closing kick of the integrator.
// FP32 mode does the geometry in FP32 from FP64 pair offsets rounded once;
// segment pairs that are nearly parallel (sin^2 < 1e-2) and near the cutoff
// are redone in FP64, because their closest points are ill-conditioned in
// FP32 (error ~ eps / sin).
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
template <typename T, typename U>
__device__ inline V3<T> cvt(V3<U> a) { return {(T)a.x, (T)a.y, (T)a.z}; }

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

// q / d for 0 <= q < 2^16 and 1 <= d <= 64 with a precomputed 1/d: the
// fractional part of (q + 1/2)/d lies in [1/(2d), 1 - 1/(2d)], far from the
// rounding error of one FP32 multiply, so truncation is exact.
__device__ inline int qdiv(int q, float inv_d) { return (int)(((float)q + 0.5f) * inv_d); }

// Nearest point of the closed segment a + t u (t in [0,1]) to p.
template <typename T>
__device__ inline V3<T> seg_point(V3<T> p, V3<T> a, V3<T> u, T inv_uu)
{
    return a + clamp01(dot(p - a, u) * inv_uu) * u;
}

// Nearest point of face f of shape S to p, both in S's body frame: the
// projection if it is inside the closed polygon (in-plane half-spaces for
// convex faces, crossing number for concave ones), else the nearest point of
// the face's own boundary edges.
template <typename T>
__device__ inline V3<T> face_point(const ShapeTab<T> &S, int f, V3<T> p)
{
    const V3<T> n = ld3(S.fn[f]);
    const T sd = dot(n, p) - S.fo[f];
    const int k0 = S.foff[f], k1 = S.foff[f + 1];
    bool inside;
    if (S.fconvex[f]) {
        inside = true;
        for (int k = k0; k < k1; ++k) inside = inside && (dot(ld3(S.lnrm[k]), p) >= S.loff[k]);
    } else {
        const V3<T> e1 = ld3(S.fe1[f]);
        const V3<T> e2 = cross(n, e1);
        const V3<T> o = ld3(S.v[S.floop[k0]]);
        const T px = dot(p - o, e1), py = dot(p - o, e2);
        inside = false;
        for (int k = k0; k < k1; ++k) {
            const int kn = (k + 1 < k1) ? k + 1 : k0;
            const T ax = S.lxy[k][0], ay = S.lxy[k][1], bx = S.lxy[kn][0], by = S.lxy[kn][1];
            if ((ay > py) != (by > py)) {
                const T xc = ax + (py - ay) * (bx - ax) / (by - ay);
                if (px < xc) inside = !inside;
            }
        }
    }
    if (inside) return p - sd * n;
    T best = T(3.0e38);
    V3<T> q = p;
    for (int k = k0; k < k1; ++k) {
        const int kn = (k + 1 < k1) ? k + 1 : k0;
        const V3<T> a = ld3(S.v[S.floop[k]]);
        const V3<T> c = seg_point(p, a, ld3(S.v[S.floop[kn]]) - a, S.linv[k]);
        const V3<T> d = p - c;
        const T d2 = dot(d, d);
        if (d2 < best) {
            best = d2;
            q = c;
        }
    }
    return q;
}

// Closest points of segments p1 + s d1 and p2 + t d2 (s, t in [0,1]).
// Non-parallel: the clamped line solution (Ericson, Real-Time Collision
// Detection, 2005, Sec. 5.1.9) with the cross-product form of its
// denominator.  Nearly parallel (|d1 x d2|^2 < par_s2 a e): each point is
// the midpoint of its segment's overlap with the other segment's
// projection, or the facing endpoint.  Returns |d1 x d2|^2.
template <typename T>
__device__ inline T seg_seg(V3<T> p1, V3<T> d1, T a, V3<T> p2, V3<T> d2, T e, T par_s2, V3<T> &P, V3<T> &Q)
{
    const V3<T> r = p1 - p2;
    const T b = dot(d1, d2), c = dot(d1, r), f = dot(d2, r);
    const V3<T> cr = cross(d1, d2);
    const T den = dot(cr, cr);
    T s, t;
    if (den < par_s2 * a * e) {
        const T ia = T(1) / a, ie = T(1) / e;
        const T t0 = -c * ia, t1 = (b - c) * ia;
        T lo = fmax(T(0), fmin(t0, t1)), hi = fmin(T(1), fmax(t0, t1));
        s = (lo <= hi) ? T(0.5) * (lo + hi) : (fmax(t0, t1) < T(0) ? T(0) : T(1));
        const T u0 = f * ie, u1 = (f + b) * ie;
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
    return den;
}

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double min_image(double d, double L) { return d - L * rint(d / L); }

__device__ inline unsigned long long lanes_below()
{
    const unsigned lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

constexpr int kWaves = 4;     // waves per block
constexpr int kQueue = 512;   // survivor queue entries per wave

template <typename T>
struct WaveLds {
    T vj[DEM_MAX_VERTS][3];   // j's vertices in i's frame
    T vi[DEM_MAX_VERTS][3];   // i's vertices in j's frame
    int queue[kQueue];
};

// One feature-pair problem: nearest points P on i and Q on j, in i's frame,
// returned as P and rho = P - Q.
template <typename T, int DIM>
struct Problem {
    const ShapeTab<T> &Si, &Sj;
    const WaveLds<T> &W;
    const M3<T> &Rr;
    V3<T> t;
    int nA, nB;
    float inv_nfj, inv_nfi, inv_nej;

    // conservative cull: false if no point of the two features can be within rc
    __device__ bool candidate(int q, T rc) const
    {
        if (DIM == 3) {
            if (q < nA) {  // vertex a of i against face f of j, in j's frame
                const int a = qdiv(q, inv_nfj), f = q - a * Sj.nf;
                const V3<T> p = ld3(W.vi[a]);
                const T sd = dot(ld3(Sj.fn[f]), p) - Sj.fo[f];
                const V3<T> dc = p - ld3(Sj.fc[f]);
                const T lim = Sj.frad[f] + rc;
                return fabs(sd) < rc && dot(dc, dc) < lim * lim;
            } else if (q < nA + nB) {  // vertex b of j against face f of i, in i's frame
                const int qq = q - nA, b = qdiv(qq, inv_nfi), f = qq - b * Si.nf;
                const V3<T> p = ld3(W.vj[b]);
                const T sd = dot(ld3(Si.fn[f]), p) - Si.fo[f];
                const V3<T> dc = p - ld3(Si.fc[f]);
                const T lim = Si.frad[f] + rc;
                return fabs(sd) < rc && dot(dc, dc) < lim * lim;
            } else {  // edge e of i against edge g of j: bounding spheres of the two segments
                const int qq = q - nA - nB, e = qdiv(qq, inv_nej), g = qq - e * Sj.ne;
                const V3<T> mj = T(0.5) * (ld3(W.vj[Sj.e[g][0]]) + ld3(W.vj[Sj.e[g][1]]));
                const V3<T> dm = ld3(Si.em[e]) - mj;
                const T lim = Si.eh[e] + Sj.eh[g] + rc;
                return dot(dm, dm) < lim * lim;
            }
        } else {
            if (q < nA) {  // vertex a of i against edge e of j, in j's frame
                const int a = qdiv(q, inv_nej), e = q - a * Sj.ne;
                const V3<T> dm = ld3(W.vi[a]) - ld3(Sj.em[e]);
                const T lim = Sj.eh[e] + rc;
                return dot(dm, dm) < lim * lim;
            } else {  // vertex b of j against edge e of i, in i's frame
                const int qq = q - nA, b = qdiv(qq, inv_nfi), e = qq - b * Si.ne;
                const V3<T> dm = ld3(W.vj[b]) - ld3(Si.em[e]);
                const T lim = Si.eh[e] + rc;
                return dot(dm, dm) < lim * lim;
            }
        }
    }

    // exact nearest points; returns the family (0: V_i-F_j / V_i-E_j, 1: V_j-F_i / V_j-E_i, 2: E_i-E_j)
    __device__ int solve(int q, T par_s2, V3<T> &P, V3<T> &rho, T &den) const
    {
        den = T(1);
        if (DIM == 3) {
            if (q < nA) {
                const int a = qdiv(q, inv_nfj), f = q - a * Sj.nf;
                const V3<T> p = ld3(W.vi[a]);
                P = ld3(Si.v[a]);
                rho = mul(Rr, p - face_point(Sj, f, p));  // offset formed in j's frame, then rotated
                return 0;
            } else if (q < nA + nB) {
                const int qq = q - nA, b = qdiv(qq, inv_nfi), f = qq - b * Si.nf;
                const V3<T> p = ld3(W.vj[b]);
                P = face_point(Si, f, p);
                rho = P - p;
                return 1;
            } else {
                const int qq = q - nA - nB, e = qdiv(qq, inv_nej), g = qq - e * Sj.ne;
                const V3<T> b0 = ld3(W.vj[Sj.e[g][0]]);
                const V3<T> d2 = ld3(W.vj[Sj.e[g][1]]) - b0;
                const T ee = T(1) / Sj.einv[g];
                V3<T> Q;
                den = seg_seg(ld3(Si.v[Si.e[e][0]]), ld3(Si.ed[e]), T(1) / Si.einv[e], b0, d2, ee, par_s2, P, Q) /
                      ((T(1) / Si.einv[e]) * ee);
                rho = P - Q;
                return 2;
            }
        } else {
            if (q < nA) {
                const int a = qdiv(q, inv_nej), e = q - a * Sj.ne;
                const V3<T> p = ld3(W.vi[a]);
                P = ld3(Si.v[a]);
                rho = mul(Rr, p - seg_point(p, ld3(Sj.v[Sj.e[e][0]]), ld3(Sj.ed[e]), Sj.einv[e]));
                return 0;
            } else {
                const int qq = q - nA, b = qdiv(qq, inv_nfi), e = qq - b * Si.ne;
                const V3<T> p = ld3(W.vj[b]);
                P = seg_point(p, ld3(Si.v[Si.e[e][0]]), ld3(Si.ed[e]), Si.einv[e]);
                rho = P - p;
                return 1;
            }
        }
    }
};

template <typename T>
struct Acc {
    V3<T> F, Ti, Tj;
    T U;
};

// WCA (Eq. 3-4) at interaction point P on i with offset rho = P - Q.
template <typename T>
__device__ inline int add_wca(Acc<T> &A, V3<T> P, V3<T> rho, V3<T> t, T sig2, T rc2, T eps)
{
    const T r2 = dot(rho, rho);
    if (!(r2 < rc2)) return 0;
    const T ir2 = T(1) / r2;
    const T s2 = sig2 * ir2;
    const T s6 = s2 * s2 * s2;
    const T h = T(2) * s6 - T(1);
    const T u = eps * h * h;  // 4 eps (s12 - s6) + eps without the cancellation of the shift
    const T fr = T(24) * eps * s6 * h * ir2;
    const V3<T> f = fr * rho;
    A.F = A.F + f;
    A.Ti = A.Ti + cross(P, f);
    A.Tj = A.Tj + cross(f, (P - rho) - t);  // lever of Q about j's centre (at t), force -f
    A.U += u;
    return 1;
}

template <typename T>
__device__ inline void load_rot(const T *rot, int n, int i, M3<T> &R)
{
    for (int k = 0; k < 9; ++k) R.m[k] = rot[(size_t)k * n + i];
}

template <typename T, int DIM>
__global__ void __launch_bounds__(64 * kWaves) k_pairs(SysParams p, StatePtrs s, ListPtrs l, const T *__restrict__ rot,
                                                          T *__restrict__ rec, const ShapeTab<T> *__restrict__ gtab,
                                                          const ShapeTab<double> *__restrict__ gtab64,
                                                          unsigned long long *stats)
{
    extern __shared__ __align__(16) unsigned char smem[];
    ShapeTab<T> *tab = reinterpret_cast<ShapeTab<T> *>(smem);
    WaveLds<T> *wl = reinterpret_cast<WaveLds<T> *>(smem + p.n_shapes * sizeof(ShapeTab<T>));
    {
        const int words = p.n_shapes * (int)(sizeof(ShapeTab<T>) / 4);
        const uint32_t *src = reinterpret_cast<const uint32_t *>(gtab);
        uint32_t *dst = reinterpret_cast<uint32_t *>(smem);
        for (int w = threadIdx.x; w < words; w += blockDim.x) dst[w] = src[w];
    }
    __syncthreads();

    const int lane = __lane_id();
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    WaveLds<T> &W = wl[wid];
    const int n = p.n;
    const int npairs = l.flags[FLAG_NPAIRS];
    // XCD-aware order: blocks are dealt round-robin to the 8 XCDs, so give
    // each XCD a contiguous share of the pair list (neighbouring particles
    // share one L2).
    const int G = gridDim.x;
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int per_xcd = (G + 7 - xcd) >> 3;  // blocks on this XCD
    int first_xcd_block = 0;
    for (int x = 0; x < xcd; ++x) first_xcd_block += (G + 7 - x) >> 3;
    const int vblock = first_xcd_block + slot;  // virtual block index, contiguous per XCD
    (void)per_xcd;
    const T par_s2 = (T)p.par_s2;
    const T eps = (T)p.eps;
    unsigned long long c_pairs = 0, c_feat = 0, c_in = 0, c_near = 0, c_ee = 0, c_ref = 0;

    for (int pr = vblock * kWaves + wid; pr < npairs; pr += G * kWaves) {
        const int i = l.pi[pr], j = l.pj[pr];
        T *out = rec + (size_t)pr * kRec;
        const double dx = min_image(s.x[j] - s.x[i], p.box[0]);
        const double dy = min_image(s.y[j] - s.y[i], p.box[1]);
        const double dz = (DIM == 3) ? min_image(s.z[j] - s.z[i], p.box[2]) : 0.0;
        const int si = s.sid[i], sj = s.sid[j];
        const double bound = p.R[si] + p.R[sj] + kWcaCut * (p.rad[si] + p.rad[sj]);
        if (dx * dx + dy * dy + dz * dz >= bound * bound) {
            if (lane < kRec) out[lane] = T(0);
            continue;
        }
        const ShapeTab<T> &Si = tab[si];
        const ShapeTab<T> &Sj = tab[sj];
        M3<T> Rr;
        V3<T> t;
        {
            M3<T> Ri, Rj;
            load_rot(rot, n, i, Ri);
            load_rot(rot, n, j, Rj);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    Rr.m[3 * a + b] = Ri.m[a] * Rj.m[b] + Ri.m[3 + a] * Rj.m[3 + b] + Ri.m[6 + a] * Rj.m[6 + b];
            t = mulT(Ri, v3<T>((T)dx, (T)dy, (T)dz));
        }
        const double sigd = p.rad[si] + p.rad[sj];
        const T sig2 = (T)(sigd * sigd);
        const T rc = (T)(kWcaCut * sigd);
        const T rc2 = rc * rc;

        // vertex sets across frames, one lane per vertex
        if (lane < Sj.nv) {
            const V3<T> v = t + mul(Rr, ld3(Sj.v[lane]));
            W.vj[lane][0] = v.x;
            W.vj[lane][1] = v.y;
            W.vj[lane][2] = v.z;
        } else if (lane >= 32 && lane - 32 < Si.nv) {
            const V3<T> v = mulT(Rr, ld3(Si.v[lane - 32]) - t);
            W.vi[lane - 32][0] = v.x;
            W.vi[lane - 32][1] = v.y;
            W.vi[lane - 32][2] = v.z;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        Problem<T, DIM> P{Si, Sj, W, Rr, t, 0, 0, 0.f, 0.f, 0.f};
        int total;
        if (DIM == 3) {
            P.nA = Si.nv * Sj.nf;
            P.nB = Sj.nv * Si.nf;
            total = P.nA + P.nB + Si.ne * Sj.ne;
            P.inv_nfj = 1.0f / (float)Sj.nf;
            P.inv_nfi = 1.0f / (float)Si.nf;
        } else {
            P.nA = Si.nv * Sj.ne;
            P.nB = Sj.nv * Si.ne;
            total = P.nA + P.nB;
            P.inv_nfi = 1.0f / (float)Si.ne;
        }
        P.inv_nej = 1.0f / (float)Sj.ne;
        c_pairs += 1;
        c_feat += total;

        Acc<T> A;
        A.F = A.Ti = A.Tj = v3<T>(0, 0, 0);
        A.U = T(0);
        int count = 0;
        for (int base = 0; base < total; base += 64) {
            const int q = base + lane;
            const bool keep = q < total && P.candidate(q, rc);
            const unsigned long long m = __ballot(keep);
            if (keep) W.queue[count + __popcll(m & lanes_below())] = q;
            count += __popcll(m);
            if (count > kQueue - 64 || base + 64 >= total) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                for (int k = lane; k < count; k += 64) {
                    const int qq = W.queue[k];
                    V3<T> Pt, rho;
                    T den;
                    const int fam = P.solve(qq, par_s2, Pt, rho, den);
                    c_near += fam < 2 ? 1 : 0;
                    c_ee += fam == 2 ? 1 : 0;
                    if (sizeof(T) == 4 && DIM == 3 && fam == 2 && den < T(1e-2) &&
                        dot(rho, rho) < T(1.0001) * rc2 + T(1e-3) * rc) {
                        // ill-conditioned in FP32: redo this edge pair in FP64 from FP64 geometry
                        const int q3 = qq - P.nA - P.nB, e = qdiv(q3, P.inv_nej), g = q3 - e * Sj.ne;
                        double Rd[9], Rjd[9];
                        quat_to_rot(s.qw[i], s.qx[i], s.qy[i], s.qz[i], Rd);
                        quat_to_rot(s.qw[j], s.qx[j], s.qy[j], s.qz[j], Rjd);
                        M3<double> Rrd;
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b)
                                Rrd.m[3 * a + b] = Rd[a] * Rjd[b] + Rd[3 + a] * Rjd[3 + b] + Rd[6 + a] * Rjd[6 + b];
                        M3<double> Rid;
                        for (int k9 = 0; k9 < 9; ++k9) Rid.m[k9] = Rd[k9];
                        const V3<double> dd = v3<double>(min_image(s.x[j] - s.x[i], p.box[0]),
                                                         min_image(s.y[j] - s.y[i], p.box[1]),
                                                         min_image(s.z[j] - s.z[i], p.box[2]));
                        const V3<double> td = mulT(Rid, dd);
                        const ShapeTab<double> &Di = gtab64[si];
                        const ShapeTab<double> &Dj = gtab64[sj];
                        const V3<double> b0 = td + mul(Rrd, ld3(Dj.v[Dj.e[g][0]]));
                        const V3<double> d2 = mul(Rrd, ld3(Dj.ed[g]));
                        V3<double> Pd, Qd;
                        seg_seg(ld3(Di.v[Di.e[e][0]]), ld3(Di.ed[e]), 1.0 / Di.einv[e], b0, d2, 1.0 / Dj.einv[g],
                                p.par_s2, Pd, Qd);
                        Pt = cvt<T>(Pd);
                        rho = cvt<T>(Pd - Qd);
                        c_ref += 1;
                    }
                    c_in += add_wca(A, Pt, rho, t, sig2, rc2, eps);
                }
                count = 0;
                __builtin_amdgcn_wave_barrier();
            }
        }
        // reduce in FP64; lane 0 rotates to the space frame and writes the record
        double F[3] = {wave_sum((double)A.F.x), wave_sum((double)A.F.y), wave_sum((double)A.F.z)};
        double Ti[3] = {wave_sum((double)A.Ti.x), wave_sum((double)A.Ti.y), wave_sum((double)A.Ti.z)};
        double Tj[3] = {wave_sum((double)A.Tj.x), wave_sum((double)A.Tj.y), wave_sum((double)A.Tj.z)};
        const double U = wave_sum((double)A.U);
        if (lane == 0) {
            M3<T> Ri;
            load_rot(rot, n, i, Ri);
            for (int a = 0; a < 3; ++a) {
                out[a] = (T)(Ri.m[3 * a] * F[0] + Ri.m[3 * a + 1] * F[1] + Ri.m[3 * a + 2] * F[2]);
                out[3 + a] = (T)(Ri.m[3 * a] * Ti[0] + Ri.m[3 * a + 1] * Ti[1] + Ri.m[3 * a + 2] * Ti[2]);
                out[6 + a] = (T)(Ri.m[3 * a] * Tj[0] + Ri.m[3 * a + 1] * Tj[1] + Ri.m[3 * a + 2] * Tj[2]);
            }
            out[9] = (T)U;
        }
    }
    if (stats) {
        unsigned long long in_w = c_in, near_w = c_near, ee_w = c_ee, ref_w = c_ref;
        for (int off = 32; off > 0; off >>= 1) {
            in_w += __shfl_xor(in_w, off, 64);
            near_w += __shfl_xor(near_w, off, 64);
            ee_w += __shfl_xor(ee_w, off, 64);
            ref_w += __shfl_xor(ref_w, off, 64);
        }
        if (lane == 0) {
            atomicAdd(&stats[ST_PAIRS], c_pairs);
            atomicAdd(&stats[ST_FEATURES], c_feat);
            atomicAdd(&stats[ST_INCUT], in_w);
            atomicAdd(&stats[ST_NEAR], near_w);
            atomicAdd(&stats[ST_REFINED], ref_w);
            atomicAdd(&stats[ST_EENEAR], ee_w);
            if (blockIdx.x == 0 && wid == 0) atomicAdd(&stats[ST_LAUNCHES], 1ull);
        }
    }
}

__device__ inline void body_torque(const double q[4], double tx, double ty, double tz, double out[3])
{
    double R[9];
    quat_to_rot(q[0], q[1], q[2], q[3], R);
    out[0] = R[0] * tx + R[3] * ty + R[6] * tz;
    out[1] = R[1] * tx + R[4] * ty + R[7] * tz;
    out[2] = R[2] * tx + R[5] * ty + R[8] * tz;
}

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
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Per-particle sums of the pair records in row order; optional closing kick.
template <typename T, int DIM, bool KICK, bool NVT>
__global__ void __launch_bounds__(kBlock) k_gather(SysParams p, StatePtrs s, OutPtrs o, ListPtrs l,
                                                      const T *__restrict__ rec, double *ke_part, double *th)
{
    __shared__ double sh[kBlock];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && l.flags[FLAG_REBUILD] != 0) {
        // the lists consumed by this step are fresh: count the build and clear the trigger
        l.flags[FLAG_REBUILD] = 0;
        l.flags[FLAG_NBUILDS] += 1;
    }
    double kt = 0.0, kr = 0.0;
    if (i < p.n) {
        const int n = p.n;
        double F[3] = {0, 0, 0}, Tq[3] = {0, 0, 0}, U = 0.0, Wm[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        const double xi = s.x[i], yi = s.y[i], zi = (DIM == 3) ? s.z[i] : 0.0;
        const int m = l.n_nbr[i];
        for (int k = 0; k < m; ++k) {
            const int j = l.nbr[(size_t)k * n + i];
            const int q = l.pidx[(size_t)k * n + i];
            if (q < 0) continue;
            const T *r = rec + (size_t)q * kRec;
            const double sg = (j > i) ? 1.0 : -1.0;  // records hold the force on the pair's owner (lower index)
            const double f[3] = {sg * (double)r[0], sg * (double)r[1], sg * (double)r[2]};
            const int to = (j > i) ? 3 : 6;
            for (int a = 0; a < 3; ++a) {
                F[a] += f[a];
                Tq[a] += (double)r[to + a];
            }
            U += 0.5 * (double)r[9];
            if (f[0] != 0.0 || f[1] != 0.0 || f[2] != 0.0) {
                const double d[3] = {min_image(s.x[j] - xi, p.box[0]), min_image(s.y[j] - yi, p.box[1]),
                                     (DIM == 3) ? min_image(s.z[j] - zi, p.box[2]) : 0.0};
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) Wm[3 * a + b] -= 0.5 * d[a] * f[b];
            }
        }
        if (DIM == 2) {
            F[2] = 0.0;
            Tq[0] = Tq[1] = 0.0;
        }
        o.Fx[i] = F[0];
        o.Fy[i] = F[1];
        o.Fz[i] = F[2];
        o.Tx[i] = Tq[0];
        o.Ty[i] = Tq[1];
        o.Tz[i] = Tq[2];
        o.U[i] = U;
        for (int c = 0; c < 9; ++c) o.W[(size_t)c * n + i] = Wm[c];
        if (KICK) {
            const int sid = s.sid[i];
            const double hm = 0.5 * p.dt / p.mass[sid];
            double v[3] = {s.vx[i] + hm * F[0], s.vy[i] + hm * F[1], 0.0};
            s.vx[i] = v[0];
            s.vy[i] = v[1];
            double L[3] = {0.0, 0.0, 0.0};
            if (DIM == 3) {
                v[2] = s.vz[i] + hm * F[2];
                s.vz[i] = v[2];
                const double q[4] = {s.qw[i], s.qx[i], s.qy[i], s.qz[i]};
                double tb[3];
                body_torque(q, Tq[0], Tq[1], Tq[2], tb);
                L[0] = s.Lx[i] + 0.5 * p.dt * tb[0];
                L[1] = s.Ly[i] + 0.5 * p.dt * tb[1];
                L[2] = s.Lz[i] + 0.5 * p.dt * tb[2];
                s.Lx[i] = L[0];
                s.Ly[i] = L[1];
                s.Lz[i] = L[2];
            } else {
                L[2] = s.Lz[i] + 0.5 * p.dt * Tq[2];
                s.Lz[i] = L[2];
            }
            if (NVT) {
                kt = 0.5 * p.mass[sid] * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                for (int a = 0; a < 3; ++a)
                    if (p.inertia[sid][a] > 0.0) kr += 0.5 * L[a] * L[a] / p.inertia[sid][a];
            }
        }
    }
    if (KICK && NVT) {
        kt = block_sum<kBlock>(kt, sh);
        kr = block_sum<kBlock>(kr, sh);
        if (threadIdx.x == 0) {
            ke_part[2 * blockIdx.x] = kt;
            ke_part[2 * blockIdx.x + 1] = kr;
            if (blockIdx.x == 0) th[TH_PENDING] = 1.0;
        }
    }
}

template <typename T>
__global__ void k_rotations(SysParams p, StatePtrs s, T *rot)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n) return;
    double R[9];
    quat_to_rot(s.qw[i], s.qx[i], s.qy[i], s.qz[i], R);
    for (int k = 0; k < 9; ++k) rot[(size_t)k * p.n + i] = (T)R[k];
}

template <typename T, int DIM>
void pairs_t(const SysParams &p, const StatePtrs &s, const ListPtrs &l, const ForcePtrs &f,
             unsigned long long *stats, hipStream_t stream)
{
    const size_t sh = (size_t)p.n_shapes * sizeof(ShapeTab<T>) + kWaves * sizeof(WaveLds<T>);
    k_pairs<T, DIM><<<p.pair_blocks, 64 * kWaves, sh, stream>>>(
        p, s, l, reinterpret_cast<const T *>(f.rot), reinterpret_cast<T *>(f.rec),
        reinterpret_cast<const ShapeTab<T> *>(f.tab), reinterpret_cast<const ShapeTab<double> *>(f.tab64), stats);
}

template <typename T, int DIM>
void gather_t(const SysParams &p, const StatePtrs &s, const OutPtrs &o, const ListPtrs &l, const ForcePtrs &f, bool kick,
              double *ke_part, double *th, hipStream_t stream)
{
    const T *rec = reinterpret_cast<const T *>(f.rec);
    const int nb = blocks_for(p.n);
    const bool nvt = p.ensemble == DEM_NVT;
    if (!kick)
        k_gather<T, DIM, false, false><<<nb, kBlock, 0, stream>>>(p, s, o, l, rec, ke_part, th);
    else if (nvt)
        k_gather<T, DIM, true, true><<<nb, kBlock, 0, stream>>>(p, s, o, l, rec, ke_part, th);
    else
        k_gather<T, DIM, true, false><<<nb, kBlock, 0, stream>>>(p, s, o, l, rec, ke_part, th);
}

}  // namespace

void launch_rotations(const SysParams &p, const StatePtrs &s, void *rot, int precision, hipStream_t stream)
{
    if (p.n == 0) return;
    if (precision == DEM_FP32)
        k_rotations<float><<<blocks_for(p.n), kBlock, 0, stream>>>(p, s, reinterpret_cast<float *>(rot));
    else
        k_rotations<double><<<blocks_for(p.n), kBlock, 0, stream>>>(p, s, reinterpret_cast<double *>(rot));
}

void launch_pairs(const SysParams &p, const StatePtrs &s, const ListPtrs &l, const ForcePtrs &f, int precision,
                  unsigned long long *stats, hipStream_t stream)
{
    if (p.n == 0) return;
    if (precision == DEM_FP32) {
        if (p.dim == 3) pairs_t<float, 3>(p, s, l, f, stats, stream);
        else pairs_t<float, 2>(p, s, l, f, stats, stream);
    } else {
        if (p.dim == 3) pairs_t<double, 3>(p, s, l, f, stats, stream);
        else pairs_t<double, 2>(p, s, l, f, stats, stream);
    }
}

void launch_gather(const SysParams &p, const StatePtrs &s, const OutPtrs &o, const ListPtrs &l, const ForcePtrs &f,
                   int precision, bool kick, double *ke_part, double *thermo, hipStream_t stream)
{
    if (p.n == 0) return;
    if (precision == DEM_FP32) {
        if (p.dim == 3) gather_t<float, 3>(p, s, o, l, f, kick, ke_part, thermo, stream);
        else gather_t<float, 2>(p, s, o, l, f, kick, ke_part, thermo, stream);
    } else {
        if (p.dim == 3) gather_t<double, 3>(p, s, o, l, f, kick, ke_part, thermo, stream);
        else gather_t<double, 2>(p, s, o, l, f, kick, ke_part, thermo, stream);
    }
}

}  // namespace dem

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
// Mapping to gfx950:
//  1. k_pairs: each unordered pair of the half list once, in two stages.
//     The separation stage (4 lanes per pair, 16 pairs per wavefront) loads
//     the pair, drops it beyond R_i + R_j + r_cut, and tests each body's
//     vertices against the other's supporting planes; a pair separated by
//     more than r_cut has no feature pair inside the cutoff.  The rest queue
//     in LDS for the feature stage (8 or 16 lanes per pair, a tuning knob):
//     a per-feature prefilter keeps only vertices, edges and faces within
//     reach of the other body and not wholly beyond one of its supporting
//     planes, every remaining feature pair of Eq. 1/2 gets a cheap
//     conservative test (plane distance and bounding circle for
//     vertex-face; bounding spheres, then the distance of the two lines, for
//     edge-edge; bounding spheres for vertex-edge), and the survivors are
//     compacted into a per-pair LDS queue so the exact nearest-point and WCA
//     work runs on dense lanes.  The group reduces force, both torques and
//     energy in a fixed order; a pair with a feature pair inside the cutoff
//     writes one record into each particle's row slot (FP32 records in FP32
//     mode; every sum over pairs is FP64) and sets the slot's bit in the
//     particle's written-slot mask.
//  2. k_gather: each particle sums the records of its written slots in slot
//     order (deterministic) into F, tau, U_i and W_i and clears its mask,
//     optionally fused with the closing kick of the integrator;
//     k_replica_tail then closes the step of each replica (thermostat half
//     steps, budget, rebuilds).
// FP32 mode does the geometry in FP32 from FP64 pair offsets rounded once;
// problems within 1% of the cutoff, segment pairs that are nearly parallel
// (sin^2 < 1e-2) and terms whose force line passes close to a centre are
// redone in FP64, because FP32 cannot resolve them (steep force near the
// cutoff; closest points ill-conditioned, error ~ eps / sin^2; a torque that
// is a small fraction of |lever| |f|).
#include <algorithm>

#include "dem_internal.h"
#include "dem_listbuild.h"

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
// the face's own boundary edges.  The face's loop (foff, floop, fconvex) is
// read from `top`, a table of the same shape that may sit in faster memory
// than S (the FP32 table in LDS beside the FP64 one in global memory); the
// loops are unrolled and free of early exits, so the loads of a face's
// loop entries are issued together instead of one round trip each.
template <typename T, typename TT>
__device__ inline V3<T> face_point(const TT &top, const ShapeTab<T> &S, int f, V3<T> p)
{
    // unrolled where S is in global memory or FP32 (registers allow it)
    constexpr int kU = (sizeof(T) == 8 && sizeof(TT) == sizeof(ShapeTab<T>)) ? 1 : 4;
    const V3<T> n = ld3(S.fn[f]);
    const T sd = dot(n, p) - S.fo[f];
    const int k0 = top.foff[f], k1 = top.foff[f + 1];
    bool inside;
    if (top.fconvex[f]) {
        inside = true;
#pragma unroll kU
        for (int k = k0; k < k1; ++k) inside &= dot(ld3(S.lnrm[k]), p) >= S.loff[k];
    } else {
        const V3<T> e1 = ld3(S.fe1[f]);
        const V3<T> e2 = cross(n, e1);
        const V3<T> o = ld3(S.v[top.floop[k0]]);
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
#pragma unroll kU
    for (int k = k0; k < k1; ++k) {
        const int kn = (k + 1 < k1) ? k + 1 : k0;
        const V3<T> a = ld3(S.v[top.floop[k]]);
        const V3<T> c = seg_point(p, a, ld3(S.v[top.floop[kn]]) - a, S.linv[k]);
        const V3<T> d = p - c;
        const T d2 = dot(d, d);
        if (d2 < best) {
            best = d2;
            q = c;
        }
    }
    return q;
}

__device__ inline double min_image(double d, double L) { return d - L * rint(d / L); }
// The same for |d| < L (positions in [0, L)) without a division; it differs
// from min_image only where |d| is within rounding of L/2, far beyond any
// interaction.
__device__ inline double min_image_near(double d, double L)
{
    const double h = 0.5 * L;
    return d > h ? d - L : (d < -h ? d + L : d);
}

// Hamilton product a b of quaternions (w, x, y, z), and the rotation of v by
// a unit quaternion q = (w, u): v + 2 w (u x v) + 2 u x (u x v).
__device__ inline void qmul(const double a[4], const double b[4], double o[4])
{
    o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}
__device__ inline V3<double> qrot(const double q[4], V3<double> v)
{
    const V3<double> u = v3<double>(q[1], q[2], q[3]);
    const V3<double> c = cross(u, v);
    return v + (2.0 * q[0]) * c + 2.0 * cross(u, c);
}

// Set bits of m in the lanes below this one (the hardware's masked bit
// count: no lane mask is held in registers).
__device__ inline int popc_below(unsigned long long m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

constexpr int kWaves = kPairWaves;  // waves per block
constexpr int kQueue = 128;        // survivor queue entries per pair
// Problem k of a solve round adds into partial sum k % kVirt, whatever the
// number of lanes per pair, and the partial sums are combined by one fixed
// tree: the result of a pair is the same bit for bit with 8 or 16 lanes.
constexpr int kVirt = 16;

// Reciprocal: the hardware FP32 estimate (1 ulp), exact division in FP64.
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp(double x) { return 1.0 / x; }

template <typename T>
struct PairLds {
    T vj[DEM_MAX_VERTS][3];   // j's vertices in i's frame
    T vi[DEM_MAX_VERTS][3];   // i's vertices in j's frame
    // features that can reach the other body (conservative prefilter), by index
    unsigned char vi_near[DEM_MAX_VERTS], vj_near[DEM_MAX_VERTS];
    unsigned char ei_near[DEM_MAX_EDGES], ej_near[DEM_MAX_EDGES];
    unsigned char fi_near[DEM_MAX_FACES], fj_near[DEM_MAX_FACES];
    // supporting planes of the other body that each vertex lies more than
    // r_cut beyond (bit p: plane p)
    unsigned vib[DEM_MAX_VERTS], vjb[DEM_MAX_VERTS];
    unsigned short queue[kQueue];
    // the pair's problem counts and queue length, for the lanes of other
    // groups that solve its problems in the pooled solve (16 lanes per pair)
    int nA, nB, nfj, nfi, nej, cnt;
};

// Feature-cell form of the feature search (one per lane group, beside its
// PairLds): the cell masks of i's edges (edges of j within reach of each,
// 3D), and the prefix of the problem counts over the near entries (i's
// vertices, j's vertices, i's edges), which numbers the pair's problems.
struct PairFc {
    unsigned eib[DEM_MAX_EDGES];
    unsigned short pf[2 * DEM_MAX_VERTS + DEM_MAX_EDGES + 2];
};

// The masks of the shape-local feature cell of shape S (its cells at
// `cells`) that holds point p, given in S's frame; zero outside the grid.
template <typename T, int DIM>
__device__ inline uint2 fc_lookup(const uint2 *__restrict__ cells, const ShapeTab<T> &S, V3<T> p)
{
    const int g = S.fc_g;
    const int ix = (int)floor((p.x - S.fc_lo) * S.fc_ih);
    const int iy = (int)floor((p.y - S.fc_lo) * S.fc_ih);
    const int iz = DIM == 3 ? (int)floor((p.z - S.fc_lo) * S.fc_ih) : 0;
    if (ix < 0 || ix >= g || iy < 0 || iy >= g || iz < 0 || iz >= (DIM == 3 ? g : 1)) return make_uint2(0u, 0u);
    return cells[(iz * g + iy) * g + ix];
}

// Index of the r-th set bit of m (r < popcount(m)).
__device__ inline int nth_bit(unsigned m, int r)
{
    for (int k = 0; k < r; ++k) m &= m - 1u;
    return __builtin_ctz(m);
}

// Closest points of segments p1 + s d1 and p2 + t d2 (s, t in [0,1]) with
// a = |d1|^2, e = |d2|^2 and their reciprocals ia, ie given.
// Non-parallel: the clamped line solution (Ericson, Real-Time Collision
// Detection, 2005, Sec. 5.1.9) with the cross-product form of its
// denominator.  Nearly parallel (|d1 x d2|^2 < par_s2 a e): each point is
// the midpoint of its segment's overlap with the other segment's
// projection, or the facing endpoint.  Returns |d1 x d2|^2.
template <typename T>
__device__ inline T seg_seg(V3<T> p1, V3<T> d1, T a, T ia, V3<T> p2, V3<T> d2, T e, T ie, T par_s2, V3<T> &P,
                            V3<T> &Q)
{
    const V3<T> r = p1 - p2;
    const T b = dot(d1, d2), c = dot(d1, r), f = dot(d2, r);
    const V3<T> cr = cross(d1, d2);
    const T den = dot(cr, cr);
    T s, t;
    if (den < par_s2 * a * e) {
        const T t0 = -c * ia, t1 = (b - c) * ia;
        T lo = fmax(T(0), fmin(t0, t1)), hi = fmin(T(1), fmax(t0, t1));
        s = (lo <= hi) ? T(0.5) * (lo + hi) : (fmax(t0, t1) < T(0) ? T(0) : T(1));
        const T u0 = f * ie, u1 = (f + b) * ie;
        lo = fmax(T(0), fmin(u0, u1));
        hi = fmin(T(1), fmax(u0, u1));
        t = (lo <= hi) ? T(0.5) * (lo + hi) : (fmax(u0, u1) < T(0) ? T(0) : T(1));
    } else {
        s = clamp01((b * f - c * e) * rcp(den));
        t = (b * s + f) * ie;
        if (t < T(0)) {
            t = T(0);
            s = clamp01(-c * ia);
        } else if (t > T(1)) {
            t = T(1);
            s = clamp01((b - c) * ia);
        }
    }
    P = p1 + s * d1;
    Q = p2 + t * d2;
    return den;
}

// The feature-pair problems of one particle pair, restricted to the
// features that passed the prefilter: family A pairs near vertices of i
// with near faces (2D: edges) of j, family B near vertices of j with near
// faces (edges) of i, family C near edges of i with near edges of j (3D).
// Problem q decodes to list positions by an exact small division.
template <typename T, int DIM, bool FC = false>
struct Problem {
    const ShapeTab<T> &Si, &Sj;
    const PairLds<T> &W;
    const M3<T> &Rr;
    V3<T> t;
    int nA, nB;
    int nfj, nfi, nej;            // list lengths used as divisors
    float inv_fj, inv_fi, inv_ej;
    // feature cells: nA, nB the near vertices of i and of j, nfj all near
    // entries (with i's near edges); problem q belongs to the entry e with
    // pf[e] <= q < pf[e + 1] and is the (q - pf[e])-th feature of its mask.
    // In both numberings the cull and the solves take the problem's code
    // fam << 10 | x << 5 | y (fc_code, pack).
    const PairFc *F = nullptr;

    __device__ int fc_code(int q) const
    {
        {
            int lo = 0, hi = nfj;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if ((int)F->pf[mid] <= q) lo = mid;
                else hi = mid;
            }
            const int r = q - (int)F->pf[lo];
            unsigned m;
            int fam, x;
            if (lo < nA) {
                fam = 0;
                x = W.vi_near[lo];
                m = W.vib[x];
            } else if (lo < nA + nB) {
                fam = 1;
                x = W.vj_near[lo - nA];
                m = W.vjb[x];
            } else {
                fam = 2;
                x = W.ei_near[lo - nA - nB];
                m = F->eib[x];
            }
            return fam << 10 | x << 5 | nth_bit(m, r);
        }
    }

    // the queue holds codes fam << 10 | x << 5 | y (the cull forms them: a
    // solve step then decodes its problem without LDS loads)
    __device__ static void decode(int code, int &fam, int &x, int &y)
    {
        fam = code >> 10;
        x = (code >> 5) & 31;
        y = code & 31;
    }

    // code of problem q of the plane-prefilter numbering: vertex x of i
    // against face (2D: edge) y of j for q < nA, vertex x of j against face
    // y of i for q < nA + nB, edge x of i against edge y of j after that
    __device__ int pack(int q) const
    {
        int fam, x, y;
        if (q < nA) {
            const int ax = qdiv(q, inv_fj);
            fam = 0;
            x = W.vi_near[ax];
            y = (DIM == 3) ? W.fj_near[q - ax * nfj] : W.ej_near[q - ax * nfj];
        } else if (q < nA + nB) {
            const int qq = q - nA, bx = qdiv(qq, inv_fi);
            fam = 1;
            x = W.vj_near[bx];
            y = (DIM == 3) ? W.fi_near[qq - bx * nfi] : W.ei_near[qq - bx * nfi];
        } else {
            const int qq = q - nA - nB, ex = qdiv(qq, inv_ej);
            fam = 2;
            x = W.ei_near[ex];
            y = W.ej_near[qq - ex * nej];
        }
        return fam << 10 | x << 5 | y;
    }

    // conservative cull: false if no point of the two features can be within rc
    __device__ bool candidate(int q, T rc) const
    {
        int fam, x, y;
        decode(q, fam, x, y);
        if (DIM == 3) {
            if (fam < 2) {  // vertex against face, in the face owner's frame
                const ShapeTab<T> &S = fam == 0 ? Sj : Si;
                const V3<T> pt = fam == 0 ? ld3(W.vi[x]) : ld3(W.vj[x]);
                const T sd = dot(ld3(S.fn[y]), pt) - S.fo[y];
                const V3<T> dc = pt - ld3(S.fc[y]);
                const T lim = S.frad[y] + rc;
                return fabs(sd) < rc && dot(dc, dc) < lim * lim;
            }
            // edge against edge: bounding spheres of the two segments, then,
            // unless they are close to parallel, the distance between their
            // lines (a lower bound of the segments' distance)
            const V3<T> a = ld3(W.vj[Sj.e[y][0]]), d2 = ld3(W.vj[Sj.e[y][1]]) - a;
            const V3<T> dm = ld3(Si.em[x]) - (a + T(0.5) * d2);
            const T lim = Si.eh[x] + Sj.eh[y] + rc;
            if (!(dot(dm, dm) < lim * lim)) return false;
            const V3<T> d1 = ld3(Si.ed[x]);
            const V3<T> n = cross(d1, d2);
            const T nn = dot(n, n);
            const T rn = dot(ld3(Si.em[x]) - a, n);
            return !(nn > T(1e-4) * Si.el2[x] * dot(d2, d2) && rn * rn > T(1.001) * rc * rc * nn);
        } else {  // vertex against edge, in the edge owner's frame
            const ShapeTab<T> &S = fam == 0 ? Sj : Si;
            const V3<T> dm = (fam == 0 ? ld3(W.vi[x]) : ld3(W.vj[x])) - ld3(S.em[y]);
            const T lim = S.eh[y] + rc;
            return dot(dm, dm) < lim * lim;
        }
    }

    // exact nearest points: P on i and rho = P - Q, in i's frame; for edge
    // pairs also sin^2 of their angle (1 otherwise)
    __device__ int solve(int q, T par_s2, V3<T> &P, V3<T> &rho, T &sin2, int &ex, int &ey) const
    {
        int fam, x, y;
        decode(q, fam, x, y);
        ex = x;
        ey = y;
        sin2 = T(1);
        if (fam == 0) {
            const V3<T> pt = ld3(W.vi[x]);
            P = ld3(Si.v[x]);
            const V3<T> qj = (DIM == 3) ? face_point(Sj, Sj, y, pt)
                                        : seg_point(pt, ld3(Sj.v[Sj.e[y][0]]), ld3(Sj.ed[y]), Sj.einv[y]);
            rho = mul(Rr, pt - qj);  // offset formed in j's frame, then rotated
        } else if (fam == 1) {
            const V3<T> pt = ld3(W.vj[x]);
            P = (DIM == 3) ? face_point(Si, Si, y, pt) : seg_point(pt, ld3(Si.v[Si.e[y][0]]), ld3(Si.ed[y]), Si.einv[y]);
            rho = P - pt;
        } else {
            const V3<T> b0 = ld3(W.vj[Sj.e[y][0]]);
            const V3<T> d2 = ld3(W.vj[Sj.e[y][1]]) - b0;
            V3<T> Q;
            const T den = seg_seg(ld3(Si.v[Si.e[x][0]]), ld3(Si.ed[x]), Si.el2[x], Si.einv[x], b0, d2, Sj.el2[y],
                                  Sj.einv[y], par_s2, P, Q);
            sin2 = den * Si.einv[x] * Sj.einv[y];
            rho = P - Q;
        }
        return fam;
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
    const T ir2 = rcp(r2);
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

// Sum over the GL lanes of a group of the lanes' two partial sums (a, b):
// partial sum s of the kVirt canonical ones is a of lane s (s < GL) or b of
// lane s - GL; the tree pairs s with s + 8 first, then halves.
template <int GL, typename T>
__device__ inline T group_sum(T a, T b)
{
    T v = GL == kVirt ? a : a + b;
    for (int off = (GL == kVirt ? kVirt / 2 : GL / 2); off > 0; off >>= 1) v += __shfl_xor(v, off, GL);
    return v;
}

__device__ inline void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Appends this lane's item to its group's list when keep is set; returns
// the group's new length.  All 64 lanes must call it together.
__device__ inline int group_append(bool keep, unsigned char *list, int len, int item, unsigned long long gmask)
{
    const unsigned long long m = __ballot(keep);
    if (keep) list[len + popc_below(m & gmask)] = (unsigned char)item;
    return len + __popcll(m & gmask);
}

// Whether FP32 cannot resolve a feature-pair problem, which is then redone
// in FP64 (refine_pair) from the FP64 positions and orientations.  P is the
// nearest point on i, rho = P - Q, t is j's centre, all in i's frame.
//  * Within 1% of the cutoff: the force is a steep function of the distance
//    (dF/dr = 72 eps / r_cut^2) and an isolated contact there has nothing to
//    hide behind.
//  * Nearly parallel edges (sin^2 < 1e-2): their closest points are
//    ill-conditioned (error ~ eps / sin^2), and the error reaches the lever.
//  * A force line that passes close to either centre (the angle between
//    rho and the lever P, or Q - t, has sin^2 < 1e-2): the term's torque is
//    then a small fraction of |lever| |f|, while the rounding of the pair
//    offset to FP32 turns the force's direction by about 1e-6, an error of
//    1e-6 |lever| |f| that would dominate it.  Bodies touching along the
//    line of their centres (a vertex on its symmetry axis, a face contact
//    centred under the other body) have zero torque this way.
template <typename T, int DIM>
__device__ inline bool fp32_unresolved(int fam, T r2, T rc2, T rc, T sin2, V3<T> P, V3<T> rho, V3<T> t)
{
    if (sizeof(T) != 4) return false;
    if (r2 > T(0.99) * rc2 && r2 < T(1.0001) * rc2) return true;
    if (DIM == 3 && fam == 2 && sin2 < T(1e-2) && r2 < T(1.0001) * rc2 + T(1e-3) * rc) return true;
    if (!(r2 < rc2)) return false;
    const V3<T> ci = cross(P, rho);
    const V3<T> lj = (P - rho) - t;
    const V3<T> cj = cross(lj, rho);
    const T k2 = T(1e-2) * r2;
    return dot(ci, ci) < k2 * dot(P, P) || dot(cj, cj) < k2 * dot(lj, lj);
}

// FP64 redo of one FP32 feature-pair problem and of its WCA terms, added to
// A: family 0 is vertex x of i against face (2D: edge) y of j, family 1
// vertex x of j against face (edge) y of i, family 2 edge x of i against
// edge y of j.  It is used where FP32 cannot resolve the answer: within 1%
// of the cutoff, where the force is a steep function of the distance
// (dF/dr = 72 eps / r_cut^2 there), and for nearly parallel edges, whose
// closest points are ill-conditioned (error ~ eps / sin).  Returns 1 if the
// pair is inside the cutoff.  Indices (edge ends, face loops) are read from
// the FP32 tables Ti, Tj in LDS, coordinates from the FP64 tables Di, Dj.
template <typename T, int DIM>
__device__ int refine_pair(const double *box, double eps, double par_s2, const PartRec64 &ri, const PartRec64 &rj,
                           const ShapeTab<T> &Ti, const ShapeTab<T> &Tj, const ShapeTab<double> &Di,
                           const ShapeTab<double> &Dj, int fam, int x, int y, double sig, Acc<T> &A)
{
    // the pair's transform as quaternions, which keeps few values live:
    // qr = conj(q_i) q_j takes j's body frame to i's, td = conj(q_i) d is
    // j's centre in i's frame
    const double qi[4] = {ri.qw, -ri.qx, -ri.qy, -ri.qz};
    const double qj[4] = {rj.qw, rj.qx, rj.qy, rj.qz};
    double qr[4];
    qmul(qi, qj, qr);
    const double qrc[4] = {qr[0], -qr[1], -qr[2], -qr[3]};
    const V3<double> dd = v3<double>(min_image_near(rj.x - ri.x, box[0]), min_image_near(rj.y - ri.y, box[1]),
                                     DIM == 3 ? min_image_near(rj.z - ri.z, box[2]) : 0.0);
    const V3<double> td = qrot(qi, dd);
    V3<double> P, rho;
    if (fam == 0) {
        const V3<double> pt = qrot(qrc, ld3(Di.v[x]) - td);  // i's vertex in j's frame
        const V3<double> q = (DIM == 3) ? face_point(Tj, Dj, y, pt)
                                        : seg_point(pt, ld3(Dj.v[Tj.e[y][0]]), ld3(Dj.ed[y]), Dj.einv[y]);
        P = ld3(Di.v[x]);
        rho = qrot(qr, pt - q);
    } else if (fam == 1) {
        const V3<double> pt = td + qrot(qr, ld3(Dj.v[x]));  // j's vertex in i's frame
        P = (DIM == 3) ? face_point(Ti, Di, y, pt) : seg_point(pt, ld3(Di.v[Ti.e[y][0]]), ld3(Di.ed[y]), Di.einv[y]);
        rho = P - pt;
    } else {
        const V3<double> b0 = td + qrot(qr, ld3(Dj.v[Tj.e[y][0]]));
        const V3<double> d2 = qrot(qr, ld3(Dj.ed[y]));
        V3<double> Q;
        seg_seg(ld3(Di.v[Ti.e[x][0]]), ld3(Di.ed[x]), Di.el2[x], Di.einv[x], b0, d2, Dj.el2[y], Dj.einv[y], par_s2,
                P, Q);
        rho = P - Q;
    }
    const double rc = kWcaCut * sig;
    Acc<double> B;
    B.F = B.Ti = B.Tj = v3<double>(0, 0, 0);
    B.U = 0.0;
    const int hit = add_wca(B, P, rho, td, sig * sig, rc * rc, eps);
    if (hit) {
        A.F = A.F + cvt<T>(B.F);
        A.Ti = A.Ti + cvt<T>(B.Ti);
        A.Tj = A.Tj + cvt<T>(B.Tj);
        A.U += (T)B.U;
    }
    return hit;
}

// The current replica of a pair-kernel block, staged in LDS beside its
// shape tables.
struct alignas(16) RepLds {
    double box[3];
    double R[DEM_MAX_SHAPES], rad[DEM_MAX_SHAPES];
    double eps, par_s2;
    int r, sbase, np, poff, first_tile, ncmp, last, pad;
};

// Stages replica r: its shape tables and parameters.  Every thread of the
// block calls it together.  UNITS: the block walks force units of the
// replica's compacted pairs (split form) instead of its pair tiles.
template <typename T, bool UNITS = false>
__device__ void stage_replica(const SysParams *reps, const ListPtrs &l, const ShapeTab<T> *gtab, ShapeTab<T> *tab,
                              RepLds &rl, int r)
{
    __syncthreads();
    const SysParams &p = reps[r];
    // 16-byte words (the tables are 16-byte aligned and sized), up to four
    // loads per thread in flight before their stores
    constexpr int kU = 4;
    const int n16 = p.n_shapes * (int)(sizeof(ShapeTab<T>) / 16);
    const uint4 *src = reinterpret_cast<const uint4 *>(gtab + p.sbase);
    uint4 *dst = reinterpret_cast<uint4 *>(tab);
    int tid = threadIdx.x;  // (formed here, not held across the caller's loop)
    asm volatile("" : "+v"(tid));
    for (int w0 = tid; w0 < n16; w0 += kU * blockDim.x) {
        uint4 v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int w = w0 + u * (int)blockDim.x;
            v[u] = w < n16 ? src[w] : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int w = w0 + u * (int)blockDim.x;
            if (w < n16) dst[w] = v[u];
        }
    }
    if (threadIdx.x == 0) {  // (one thread: the LDS addresses stay scalar)
        for (int k = 0; k < DEM_MAX_SHAPES; ++k) {
            rl.R[k] = p.R[k];
            rl.rad[k] = p.rad[k];
        }
        for (int a = 0; a < 3; ++a) rl.box[a] = p.box[a];
        rl.eps = p.eps;
        rl.par_s2 = p.par_s2;
        rl.r = r;
        rl.sbase = p.sbase;
        rl.np = l.flags[r * FLAG_COUNT + FLAG_NPAIRS];
        rl.poff = p.poff;
        rl.first_tile = UNITS ? l.cunit[r] : l.tile_start[r];
        rl.ncmp = UNITS ? l.ccount[r] : 0;
    }
    __syncthreads();
}

// j's body frame in i's, R_i^T R_j (rows of R are body axes in space).
template <typename T>
__device__ inline M3<T> rel_rotation(const M3<T> &Ri, const M3<T> &Rj)
{
    M3<T> Rr;
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c)
            Rr.m[3 * a + c] = Ri.m[a] * Rj.m[c] + Ri.m[3 + a] * Rj.m[3 + c] + Ri.m[6 + a] * Rj.m[6 + c];
    return Rr;
}

// A live pair that no supporting plane separates, parked in its wave's LDS
// queue until the wave holds one for each of its groups.
template <typename T>
struct alignas(16) QEnt {
    int4 ent;    // i, j, slot of j in row i, slot of i in row j (-1: none)
    int si, sj, pad0, pad1;
    T Rr[9];     // R_i^T R_j: j's body frame in i's
    T t[3];      // R_i^T d: j's centre in i's frame
    T Ri[9];     // R_i, body to space
    T d[3];      // minimum-image x_j - x_i
};
// The separation stage takes SL lanes per pair, so a wavefront settles
// 64 / SL pairs at a time whatever the feature stage's lane count; a tile
// is kPairWaves * 64 / SL pairs.
// queue slots per wave: one separation tile adds at most 64 / SL
// entries to fewer than one per feature-stage group already waiting
constexpr int queue_slots(int sep, int lanes) { return 64 / sep + 64 / lanes; }

// One block of 4 waves takes a contiguous range of tiles (64 or 16 pairs
// of one replica each; wave w takes pairs (64 / SL) w .. (64 / SL)(w + 1)
// - 1 of a tile in the first stage).
// Blocks are dealt round-robin to the 8 XCDs, so block b runs on XCD b % 8:
// XCD x gets the x-th eighth of the tiles, and pairs of neighbouring
// particles share its L2.  The tables of the block's current replica live
// in LDS and are restaged when its range crosses into the next replica.
//
// A pair passes two stages.  The first loads it and tests it against the
// bound R_i + R_j + r_cut and against the supporting planes of both bodies:
// when every vertex of one body lies more than r_cut beyond a supporting
// plane of the other, the two inner bodies are farther apart than r_cut, no
// feature pair of Eq. 1/2 is inside the cutoff, and the pair's record is
// zero (4 lanes per pair, 16 pairs per wavefront).  The other live pairs
// wait in the wave's LDS queue; whenever it holds one for each group of the
// second stage (GL lanes per pair; or the range or the replica ends) that
// stage runs the feature prefilter, the per-problem cull and the exact
// solves on them, so the costly stage runs on full waves.  A pair's result
// does not depend on which group or round takes it.
// Work counter of one lane; the uncounted kernel keeps none (registers).
template <bool ON>
struct Tally {
    unsigned v = 0;
    __device__ void add(unsigned x) { v += x; }
    __device__ unsigned get() const { return v; }
};
template <>
struct Tally<false> {
    __device__ void add(unsigned) {}
    __device__ unsigned get() const { return 0; }
};

// OCC wavefronts per SIMD (2 or 3, a tuning knob): the kernel is
// latency-bound, so more resident waves overlap more round trips, but at 3
// the compiler must fit 168 registers and schedules with less freedom.  The
// uncounted variants fit without spilling because the feature stage reads
// the pair's transform from the LDS queue instead of holding it.
template <typename T, int DIM, int GL, bool COUNT, int OCC, int SL, int STAGE, bool FC>
__global__ void __launch_bounds__(64 * kWaves, OCC) k_pairs(BatchParams b, const SysParams *__restrict__ reps, StatePtrs s,
                                                          ListPtrs l, const PartRec<T> *__restrict__ prec,
                                                          const PartRec64 *__restrict__ rec64,
                                                          SlotRec<T> *__restrict__ rec, const ShapeTab<T> *__restrict__ gtab,
                                                          const ShapeTab<double> *__restrict__ gtab64,
                                                          unsigned long long *stats)
{
    static_assert(GL == 8 || GL == 16, "8 or 16 lanes per pair");
    static_assert(OCC >= 2 && OCC <= 4, "2 to 4 wavefronts per SIMD");
    static_assert(SL == 4 || SL == 16, "4 or 16 lanes per pair in the separation stage");
    static_assert(STAGE >= kFused && STAGE <= kForces, "fused, search or forces");
    constexpr bool kSearch = STAGE == kSearchOnly;  // first stage only: compact the pairs it keeps
    constexpr bool kForce = STAGE == kForces;       // second stage only, on the compacted pairs
    constexpr int kSepLanes = SL;
    constexpr int kPairsPerWave = 64 / SL;
    constexpr int kGL = GL;                                    // lanes per particle pair
    constexpr int kGroups = 64 / kGL;                         // pairs per wave in the feature stage
    constexpr int kTile = kWaves * kPairsPerWave;             // pairs per block tile
    constexpr int kQCap = queue_slots(SL, kGL);
    constexpr int kVP = (DEM_MAX_VERTS + kSepLanes - 1) / kSepLanes;  // vertices per lane in the separation test
    constexpr int kSets = kVirt / kGL;                        // partial sums per lane
    extern __shared__ __align__(16) unsigned char smem[];
    const size_t orl = b.tab_slots * sizeof(ShapeTab<T>);
    ShapeTab<T> *tab = reinterpret_cast<ShapeTab<T> *>(smem);
    RepLds &rl = *reinterpret_cast<RepLds *>(smem + orl);
    PairLds<T> *pls = reinterpret_cast<PairLds<T> *>(smem + orl + sizeof(RepLds));
    QEnt<T> *qall = reinterpret_cast<QEnt<T> *>(smem + orl + sizeof(RepLds) + kWaves * kGroups * sizeof(PairLds<T>));
    // results of one pooled solve step, one per lane (16 lanes per pair only)
    constexpr bool kPool = kGL == 16;
    Acc<T> *pres = reinterpret_cast<Acc<T> *>(reinterpret_cast<unsigned char *>(qall) + kWaves * kQCap * sizeof(QEnt<T>));
    // the feature-cell form's per-group prefix and edge masks
    PairFc *pfc = reinterpret_cast<PairFc *>(reinterpret_cast<unsigned char *>(pres) +
                                             (kPool ? kWaves * 64 * sizeof(Acc<T>) : 0));

    const int lane = __lane_id();
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int grp = lane / kGL, sub = lane % kGL;
    const unsigned long long gmask = ((kGL == 64) ? ~0ull : ((1ull << kGL) - 1)) << (kGL * grp);
    PairLds<T> &W = pls[wid * kGroups + grp];
    QEnt<T> *qb = qall + wid * kQCap;
    const size_t N = (size_t)b.N;
    const int ntiles = l.tile_start[b.nrep];
    const unsigned stamp = (unsigned)l.gflags[G_STAMP];
    const int G = gridDim.x, per = G >> 3;
    // the force kernel's units: kWaves * kGroups compacted pairs of one
    // replica, so each wavefront takes one feature round
    const int *first = kForce ? l.cunit : l.tile_start;
    const int nunits = kForce ? l.cunit[b.nrep] : ntiles;
    // XCD x (block b runs on XCD b % 8) takes the x-th eighth of the units;
    // its q-th block (q = b / 8) a contiguous share of them, or, when the
    // eighth holds fewer units than the XCD has blocks, unit q: the blocks
    // launched first take the work, and no unit waits for the grid's last
    // blocks to be dispatched
    const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
    const int us = (int)((long long)nunits * xcd / 8), un = (int)((long long)nunits * (xcd + 1) / 8) - us;
    int t0, t1;
    if (q >= per) {  // (grids are multiples of 8; none is left over)
        t0 = t1 = 0;
    } else if (un >= per) {
        t0 = us + (int)((long long)un * q / per);
        t1 = us + (int)((long long)un * (q + 1) / per);
    } else {
        t0 = us + (q < un ? q : un);
        t1 = us + (q < un ? q + 1 : un);
    }
    const T grow = T(1.00001);
    Tally<COUNT> c_pairs, c_feat, c_in, c_near, c_ee, c_ref, c_sep, c_pv;

    int r = 0, r_end = 0;
    if (t0 < t1) {  // replica of the first tile: the last r with tile_start[r] <= t0
        int lo = 0, hi = b.nrep;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (first[mid] <= t0) lo = mid;
            else hi = mid;
        }
        r = lo;
        r_end = first[r + 1];
        stage_replica<T, kForce>(reps, l, gtab, tab, rl, r);
    }
    int head = 0, tail = 0;  // queue positions, the same in every lane of the wave
    int tt = t0;
    for (;;) {
        const bool done = tt >= t1;
        const bool restage = !done && tt >= r_end;
        const int pending = tail - head;
        if (!kSearch && (pending >= kGroups || (pending > 0 && (kForce || done || restage)))) {
            // ---- second stage: group g takes queue entry head + g ----
            const int take = pending < kGroups ? pending : kGroups;
            const bool live = grp < take;
            // the entry stays in LDS for the whole round (nothing is queued
            // before the next separation tile): the transform is read from
            // there where it is used, which keeps registers free for the
            // solves and the FP64 redo
            const QEnt<T> &qe = qb[(head + grp) % kQCap];
            const M3<T> &Rr = *reinterpret_cast<const M3<T> *>(qe.Rr);
            int si = 0, sj = 0;
            V3<T> t = v3<T>(0, 0, 0);
            if (live) {
                si = qe.si;
                sj = qe.sj;
                t = v3<T>(qe.t[0], qe.t[1], qe.t[2]);
            }
            const int h0 = head;  // the round's first entry
            head += take;
            const ShapeTab<T> &Si = tab[si];
            const ShapeTab<T> &Sj = tab[sj];
            const T par_s2 = (T)rl.par_s2;
            const T eps = (T)rl.eps;
            T sig2 = T(0), rc = T(0), Bi = T(0), Bj = T(0);
            if (live) {
                const double sigd = rl.rad[si] + rl.rad[sj];
                sig2 = (T)(sigd * sigd);
                rc = (T)(kWcaCut * sigd);
                Bi = (T)rl.R[si] + rc;
                Bj = (T)rl.R[sj] + rc;
            }
            const T rc2 = rc * rc;
            const T rcm = rc * T(1.0001);  // the cull keeps pairs FP32 may place just outside the cutoff

            // Feature prefilter (conservative): a vertex, edge or face can touch
            // the other body only if it lies within R_other + r_cut of that body's
            // centre, widened by the edge half length or the face's bounding
            // radius, and if it is not wholly more than r_cut beyond one of
            // the other body's supporting planes (for an edge or a face: all
            // its vertices beyond the same plane).  One lane per feature;
            // survivors are listed by index.
            int cvj = 0, cvi = 0, cei = 0, cej = 0, cfi = 0, cfj = 0;
            int fc_total = 0;
            PairFc &Fc = pfc[FC ? wid * kGroups + grp : 0];
            const T thr = rcm + T(1e-5) * (Bi + Bj);
            for (int v0 = 0; v0 < DEM_MAX_VERTS; v0 += kGL) {
                const int vk = v0 + sub;
                bool nj = false, ni = false;
                if (live && vk < Sj.nv) {
                    const V3<T> v = t + mul(Rr, ld3(Sj.v[vk]));
                    W.vj[vk][0] = v.x;
                    W.vj[vk][1] = v.y;
                    W.vj[vk][2] = v.z;
                    unsigned mb = 0;
#pragma unroll 4
                    for (int p = 0; p < Si.nsep; ++p) mb |= (dot(ld3(Si.sn[p]), v) - Si.so[p] > thr ? 1u : 0u) << p;
                    W.vjb[vk] = mb;
                    nj = mb == 0 && dot(v, v) < grow * Bi * Bi;
                }
                if (live && vk < Si.nv) {
                    const V3<T> v = mulT(Rr, ld3(Si.v[vk]) - t);
                    W.vi[vk][0] = v.x;
                    W.vi[vk][1] = v.y;
                    W.vi[vk][2] = v.z;
                    unsigned mb = 0;
#pragma unroll 4
                    for (int p = 0; p < Sj.nsep; ++p) mb |= (dot(ld3(Sj.sn[p]), v) - Sj.so[p] > thr ? 1u : 0u) << p;
                    W.vib[vk] = mb;
                    ni = mb == 0 && dot(v, v) < grow * Bj * Bj;
                }
                cvj = group_append(nj, W.vj_near, cvj, vk, gmask);
                cvi = group_append(ni, W.vi_near, cvi, vk, gmask);
                if (__ballot(live && (v0 + kGL < Si.nv || v0 + kGL < Sj.nv)) == 0) break;
            }
            wave_sync_lds();
            for (int e0 = 0; e0 < DEM_MAX_EDGES; e0 += kGL) {
                const int e = e0 + sub;
                bool ne = false, me = false;
                if (live && e < Si.ne) {
                    const V3<T> d = ld3(Si.em[e]) - t;
                    const T lim = Bj + Si.eh[e];
                    ne = (W.vib[Si.e[e][0]] & W.vib[Si.e[e][1]]) == 0 && dot(d, d) < grow * lim * lim;
                }
                if (live && e < Sj.ne) {
                    const V3<T> m = T(0.5) * (ld3(W.vj[Sj.e[e][0]]) + ld3(W.vj[Sj.e[e][1]]));
                    const T lim = Bi + Sj.eh[e];
                    me = (W.vjb[Sj.e[e][0]] & W.vjb[Sj.e[e][1]]) == 0 && dot(m, m) < grow * lim * lim;
                }
                cei = group_append(ne, W.ei_near, cei, e, gmask);
                cej = group_append(me, W.ej_near, cej, e, gmask);
                if (__ballot(live && (e0 + kGL < Si.ne || e0 + kGL < Sj.ne)) == 0) break;
            }
            if (DIM == 3) {
                const V3<T> ti = -(T)1 * mulT(Rr, t);  // i's centre in j's frame
                for (int f0 = 0; f0 < DEM_MAX_FACES; f0 += kGL) {
                    const int f = f0 + sub;
                    bool nf = false, mf = false;
                    if (live && f < Si.nf) {
                        const V3<T> d = ld3(Si.fc[f]) - t;
                        const T lim = Bj + Si.frad[f];
                        unsigned all = ~0u;
#pragma unroll 4
                        for (int k = Si.foff[f]; k < Si.foff[f + 1]; ++k) all &= W.vib[Si.floop[k]];
                        nf = all == 0 && dot(d, d) < grow * lim * lim;
                    }
                    if (live && f < Sj.nf) {
                        const V3<T> d = ld3(Sj.fc[f]) - ti;
                        const T lim = Bi + Sj.frad[f];
                        unsigned all = ~0u;
#pragma unroll 4
                        for (int k = Sj.foff[f]; k < Sj.foff[f + 1]; ++k) all &= W.vjb[Sj.floop[k]];
                        mf = all == 0 && dot(d, d) < grow * lim * lim;
                    }
                    cfi = group_append(nf, W.fi_near, cfi, f, gmask);
                    cfj = group_append(mf, W.fj_near, cfj, f, gmask);
                    if (__ballot(live && (f0 + kGL < Si.nf || f0 + kGL < Sj.nf)) == 0) break;
                }
            }
            wave_sync_lds();
            if constexpr (FC) {
                // Shape-local feature cells narrow the near sets per feature:
                // a near vertex keeps only the other body's near faces (2D:
                // edges) listed by the cell it lies in, a near edge of i only
                // j's near edges listed by the cell of its midpoint.
                unsigned mfi = 0u, mfj = 0u, mei = 0u, mej = 0u;
                for (int k = sub; k < cfi; k += kGL) mfi |= 1u << W.fi_near[k];
                for (int k = sub; k < cfj; k += kGL) mfj |= 1u << W.fj_near[k];
                for (int k = sub; k < cei; k += kGL) mei |= 1u << W.ei_near[k];
                for (int k = sub; k < cej; k += kGL) mej |= 1u << W.ej_near[k];
                for (int off = 1; off < kGL; off <<= 1) {
                    mfi |= __shfl_xor(mfi, off, kGL);
                    mfj |= __shfl_xor(mfj, off, kGL);
                    mei |= __shfl_xor(mei, off, kGL);
                    mej |= __shfl_xor(mej, off, kGL);
                }
                const unsigned tj = DIM == 3 ? mfj : mej, ti = DIM == 3 ? mfi : mei;
                const uint2 *celli = l.fcells + (size_t)(rl.sbase + si) * kFcCells;
                const uint2 *cellj = l.fcells + (size_t)(rl.sbase + sj) * kFcCells;
                for (int k = sub; k < cvi; k += kGL) {
                    const int x = W.vi_near[k];
                    W.vib[x] = fc_lookup<T, DIM>(cellj, Sj, ld3(W.vi[x])).x & tj;
                }
                for (int k = sub; k < cvj; k += kGL) {
                    const int x = W.vj_near[k];
                    W.vjb[x] = fc_lookup<T, DIM>(celli, Si, ld3(W.vj[x])).x & ti;
                }
                if (DIM == 3)
                    for (int k = sub; k < cei; k += kGL) {
                        const int e = W.ei_near[k];
                        const V3<T> m = T(0.5) * (ld3(W.vi[Si.e[e][0]]) + ld3(W.vi[Si.e[e][1]]));
                        Fc.eib[e] = fc_lookup<T, DIM>(cellj, Sj, m).y & mej;
                    }
                wave_sync_lds();
                // problem counts of the near entries (i's vertices, j's
                // vertices, i's edges in 3D) and their prefix, GL at a time
                const int nent = cvi + cvj + (DIM == 3 ? cei : 0);
                if (sub == 0) Fc.pf[0] = 0;
                for (int k0 = 0; k0 < nent; k0 += kGL) {
                    const int k = k0 + sub;
                    int c = 0;
                    if (k < nent)
                        c = __popc(k < cvi ? W.vib[W.vi_near[k]]
                                           : (k < cvi + cvj ? W.vjb[W.vj_near[k - cvi]] : Fc.eib[W.ei_near[k - cvi - cvj]]));
                    for (int off = 1; off < kGL; off <<= 1) {
                        const int u = __shfl_up(c, off, kGL);
                        if (sub >= off) c += u;
                    }
                    if (k < nent) Fc.pf[k + 1] = (unsigned short)(fc_total + c);
                    fc_total += __shfl(c, kGL - 1, kGL);
                }
                wave_sync_lds();
            }

            Problem<T, DIM, FC> P{Si, Sj, W, Rr, t, 0, 0, 1, 1, 1, 1.f, 1.f, 1.f};
            int total;
            if (FC) {
                P.nA = cvi;
                P.nB = cvj;
                P.nfj = cvi + cvj + (DIM == 3 ? cei : 0);
                P.F = &Fc;
                total = fc_total;
            } else if (DIM == 3) {
                P.nA = cvi * cfj;
                P.nB = cvj * cfi;
                total = P.nA + P.nB + cei * cej;
                P.nfj = cfj;
                P.nfi = cfi;
            } else {
                P.nA = cvi * cej;
                P.nB = cvj * cei;
                total = P.nA + P.nB;
                P.nfj = cej;
                P.nfi = cei;
            }
            P.nej = cej;
            P.inv_fj = 1.0f / (float)(P.nfj > 0 ? P.nfj : 1);
            P.inv_fi = 1.0f / (float)(P.nfi > 0 ? P.nfi : 1);
            P.inv_ej = 1.0f / (float)(P.nej > 0 ? P.nej : 1);
            if (!live) total = 0;
            if (sub == 0 && live) c_feat.add(total);

            Acc<T> A0, A1;  // partial sums kVirt-canonical: sub and sub + GL
            A0.F = A0.Ti = A0.Tj = A1.F = A1.Ti = A1.Tj = v3<T>(0, 0, 0);
            A0.U = A1.U = T(0);
            int count = 0;
            for (int qb = 0;; qb += kGL) {
                const int q = qb + sub;
                const bool has = q < total;
                const bool last = __ballot(has) == 0;
                if (!last) {
                    const int qc = has ? (FC ? P.fc_code(q) : P.pack(q)) : 0;
                    const bool keep = has && P.candidate(qc, rcm);
                    const unsigned long long m = __ballot(keep);
                    if (keep) W.queue[count + popc_below(m & gmask)] = (unsigned short)qc;
                    count += __popcll(m & gmask);
                }
                // rounds end at the same problems for any lane count and any
                // other pairs in the wavefront: a pair's queue is checked
                // after each kVirt of its candidates, and only a pair whose
                // queue is nearly full (or every pair, after its last
                // candidate) solves it at that point
                const bool full = (qb + kGL) % kVirt == 0 && count > kQueue - kVirt;
                if (last || __ballot(full) != 0) {
                    const bool mine = last || full;  // this pair solves its queue now
                    wave_sync_lds();
                    if constexpr (kPool) {
                        // The round's problems of all the wavefront's pairs
                        // are shared out over its 64 lanes, so a pair with
                        // many problems no longer holds up the others; each
                        // result goes through LDS to the lane that owns its
                        // partial sum (problem k: lane k mod 16 of the pair's
                        // group) and is added there in problem order, the
                        // order of the unpooled steps, so every pair shape
                        // gives the same bits.
                        if (sub == 0) {
                            W.nA = P.nA;
                            W.nB = P.nB;
                            W.nfj = P.nfj;
                            W.nfi = P.nfi;
                            W.nej = P.nej;
                            W.cnt = mine ? count : 0;
                        }
                        wave_sync_lds();
                        int offs[kGroups + 1];
                        offs[0] = 0;
#pragma unroll
                        for (int h = 0; h < kGroups; ++h) offs[h + 1] = offs[h] + pls[wid * kGroups + h].cnt;
                        Acc<T> *res = pres + wid * 64;
                        for (int c0 = 0; c0 < offs[kGroups]; c0 += 64) {
                            const int c = c0 + lane;
                            Acc<T> A;
                            A.F = A.Ti = A.Tj = v3<T>(0, 0, 0);
                            A.U = T(0);
                            if (c < offs[kGroups]) {
                                int g = 0;
#pragma unroll
                                for (int h = 1; h < kGroups; ++h) g += c >= offs[h] ? 1 : 0;
                                const PairLds<T> &Wg = pls[wid * kGroups + g];
                                const QEnt<T> &qg = qall[wid * kQCap + (h0 + g) % kQCap];
                                const int gi = qg.si, gj = qg.sj;
                                const ShapeTab<T> &Sgi = tab[gi];
                                const ShapeTab<T> &Sgj = tab[gj];
                                const V3<T> tg = v3<T>(qg.t[0], qg.t[1], qg.t[2]);
                                const Problem<T, DIM, FC> Pg{Sgi, Sgj, Wg, *reinterpret_cast<const M3<T> *>(qg.Rr), tg,
                                                             Wg.nA, Wg.nB, Wg.nfj, Wg.nfi, Wg.nej,
                                                             1.0f / (float)(Wg.nfj > 0 ? Wg.nfj : 1),
                                                             1.0f / (float)(Wg.nfi > 0 ? Wg.nfi : 1),
                                                             1.0f / (float)(Wg.nej > 0 ? Wg.nej : 1)};
                                const double sigd = rl.rad[gi] + rl.rad[gj];
                                const T gsig2 = (T)(sigd * sigd);
                                const T grc = (T)(kWcaCut * sigd);
                                const T grc2 = grc * grc;
                                V3<T> Pt, rho;
                                T sin2;
                                int e, gf;
                                const int fam = Pg.solve(Wg.queue[c - offs[g]], par_s2, Pt, rho, sin2, e, gf);
                                c_near.add(fam < 2 ? 1 : 0);
                                c_ee.add(fam == 2 ? 1 : 0);
                                const T r2 = dot(rho, rho);
                                const bool redo = fp32_unresolved<T, DIM>(fam, r2, grc2, grc, sin2, Pt, rho, tg);
                                if (redo) {
                                    c_ref.add(1);
                                    c_in.add(refine_pair<T, DIM>(rl.box, rl.eps, rl.par_s2, rec64[qg.ent.x], rec64[qg.ent.y],
                                                                Sgi, Sgj, gtab64[rl.sbase + gi], gtab64[rl.sbase + gj], fam,
                                                                e, gf, sigd, A));
                                } else {
                                    c_in.add(add_wca(A, Pt, rho, tg, gsig2, grc2, eps));
                                }
                            }
                            res[lane] = A;
                            wave_sync_lds();
                            // this lane's partial sum: problems sub, sub + 16, ...
                            // of its pair that fall in this step
                            const int lo = offs[grp] > c0 ? offs[grp] : c0;
                            const int hi = offs[grp + 1] < c0 + 64 ? offs[grp + 1] : c0 + 64;
                            int k = lo - offs[grp];
                            k += (sub - k % kVirt + kVirt) % kVirt;
                            for (; offs[grp] + k < hi; k += kVirt) {
                                const Acc<T> &B = res[offs[grp] + k - c0];
                                A0.F = A0.F + B.F;
                                A0.Ti = A0.Ti + B.Ti;
                                A0.Tj = A0.Tj + B.Tj;
                                A0.U += B.U;
                            }
                            wave_sync_lds();
                        }
                    } else
                    for (int m = 0;; ++m) {
                        const int k = m * kGL + sub;
                        const bool w = mine && k < count;
                        if (__ballot(w) == 0) break;
                        if (w) {
                            Acc<T> A;
                            A.F = A.Ti = A.Tj = v3<T>(0, 0, 0);
                            A.U = T(0);
                            V3<T> Pt, rho;
                            T sin2;
                            int e, g;
                            const int fam = P.solve(W.queue[k], par_s2, Pt, rho, sin2, e, g);
                            c_near.add(fam < 2 ? 1 : 0);
                            c_ee.add(fam == 2 ? 1 : 0);
                            const T r2 = dot(rho, rho);
                            const bool redo = fp32_unresolved<T, DIM>(fam, r2, rc2, rc, sin2, Pt, rho, t);
                            if (redo) {
                                c_ref.add(1);
                                c_in.add(refine_pair<T, DIM>(rl.box, rl.eps, rl.par_s2, rec64[qe.ent.x], rec64[qe.ent.y], Si, Sj,
                                                            gtab64[rl.sbase + si], gtab64[rl.sbase + sj], fam, e, g, rl.rad[si] + rl.rad[sj], A));
                            } else {
                                c_in.add(add_wca(A, Pt, rho, t, sig2, rc2, eps));
                            }
                            Acc<T> &S = (kSets == 1 || (m & 1) == 0) ? A0 : A1;
                            S.F = S.F + A.F;
                            S.Ti = S.Ti + A.Ti;
                            S.Tj = S.Tj + A.Tj;
                            S.U += A.U;
                        }
                    }
                    if (mine) count = 0;
                    wave_sync_lds();
                }
                if (last) break;
            }
            // group reduction (every lane of the group gets the sums); rotate to
            // the space frame and write both row slots, one record per lane
            const T F0 = group_sum<kGL>(A0.F.x, A1.F.x), F1 = group_sum<kGL>(A0.F.y, A1.F.y),
                    F2 = group_sum<kGL>(A0.F.z, A1.F.z);
            const T I0 = group_sum<kGL>(A0.Ti.x, A1.Ti.x), I1 = group_sum<kGL>(A0.Ti.y, A1.Ti.y),
                    I2 = group_sum<kGL>(A0.Ti.z, A1.Ti.z);
            const T J0 = group_sum<kGL>(A0.Tj.x, A1.Tj.x), J1 = group_sum<kGL>(A0.Tj.y, A1.Tj.y),
                    J2 = group_sum<kGL>(A0.Tj.z, A1.Tj.z);
            const T U = group_sum<kGL>(A0.U, A1.U);
            if (live && sub < 2) {  // lane 0 writes i's slot, lane 1 j's
                const int4 ent = qe.ent;
                const int i = ent.x, j = ent.y;
                M3<T> Ri;
                for (int k = 0; k < 9; ++k) Ri.m[k] = qe.Ri[k];
                const V3<T> dv = v3<T>(qe.d[0], qe.d[1], qe.d[2]);
                const V3<T> Fs = mul(Ri, v3<T>(F0, F1, F2));
                const bool js = sub == 1;
                const V3<T> Ts = mul(Ri, js ? v3<T>(J0, J1, J2) : v3<T>(I0, I1, I2));
                const T sg = js ? T(-1) : T(1);
                const int slot = js ? ent.w : ent.z;
                if (slot >= 0) {
                    SlotRec<T> w;
                    w.F[0] = sg * Fs.x;
                    w.F[1] = sg * Fs.y;
                    w.F[2] = sg * Fs.z;
                    w.U = U;
                    w.tq[0] = Ts.x;
                    w.tq[1] = Ts.y;
                    w.tq[2] = Ts.z;
                    w.d[0] = sg * dv.x;
                    w.d[1] = sg * dv.y;
                    w.d[2] = sg * dv.z;
                    w.pad1 = T(0);
                    set_stamp(w, stamp);
                    const int pi = js ? j : i;
                    rec[(size_t)slot * N + pi] = w;
                    atomicOr(&l.smask[(size_t)(slot >> 5) * N + pi], 1u << (slot & 31));
                }
            }
            continue;
        }
        if (done) break;
        if (restage) {
            do {
                ++r;
                r_end = first[r + 1];
            } while (tt >= r_end);
            stage_replica<T, kForce>(reps, l, gtab, tab, rl, r);
        }
        if constexpr (kForce) {
            // ---- unit tt: this wave's kGroups compacted pairs, one lane each ----
            // (uniform over the wave: the queue positions stay scalar)
            const int base = __builtin_amdgcn_readfirstlane((tt - rl.first_tile) * (kWaves * kGroups) + wid * kGroups);
            const int left = __builtin_amdgcn_readfirstlane(rl.ncmp) - base;
            const int n = left < 0 ? 0 : (left > kGroups ? kGroups : left);
            head = tail = 0;  // the queue is empty between units
            if (lane < n) {
                const int4 ent = l.cpairs[rl.poff + base + lane];
                const PartRec<T> ri = prec[ent.x];
                const PartRec<T> rj = prec[ent.y];
                M3<T> Ri, Rj;
                for (int k = 0; k < 9; ++k) {
                    Ri.m[k] = ri.R[k];
                    Rj.m[k] = rj.R[k];
                }
                const double dx = min_image(rj.x - ri.x, rl.box[0]);
                const double dy = min_image(rj.y - ri.y, rl.box[1]);
                const double dz = (DIM == 3) ? min_image(rj.z - ri.z, rl.box[2]) : 0.0;
                const M3<T> Rr = rel_rotation(Ri, Rj);
                const V3<T> t = mulT(Ri, v3<T>((T)dx, (T)dy, (T)dz));
                QEnt<T> &e = qb[lane];
                e.ent = ent;
                e.si = ri.sid;
                e.sj = rj.sid;
                for (int k = 0; k < 9; ++k) {
                    e.Rr[k] = Rr.m[k];
                    e.Ri[k] = Ri.m[k];
                }
                e.t[0] = t.x;
                e.t[1] = t.y;
                e.t[2] = t.z;
                e.d[0] = (T)dx;
                e.d[1] = (T)dy;
                e.d[2] = (T)dz;
            }
            tail = n;
            wave_sync_lds();
            ++tt;
            continue;
        }
        // ---- first stage on tile tt: 4 lanes per pair ----
        // (lane indices formed here, not held across the feature stage: an
        // empty asm keeps the compiler from hoisting them out of the loop)
        int lane1 = lane;
        asm volatile("" : "+v"(lane1));
        const int grp1 = lane1 / kSepLanes, sub1 = lane1 % kSepLanes;
        const int q = (tt - rl.first_tile) * kTile + wid * kPairsPerWave + grp1;
        const bool active = q < rl.np;
        // two dependent round trips: the pair entry, then both particle
        // records (position, rotation and shape in one line each)
        int4 ent = make_int4(0, 0, 0, 0);
        if (active) ent = l.pairs[rl.poff + q];
        const int i = ent.x, j = ent.y;
        int si = 0, sj = 0;
        double dx = 0.0, dy = 0.0, dz = 0.0;
        bool live = false;
        M3<T> Ri, Rj;
        for (int k = 0; k < 9; ++k) Ri.m[k] = Rj.m[k] = T(0);
        if (active) {
            const PartRec<T> ri = prec[i];
            const PartRec<T> rj = prec[j];
            for (int k = 0; k < 9; ++k) {
                Ri.m[k] = ri.R[k];
                Rj.m[k] = rj.R[k];
            }
            dx = min_image(rj.x - ri.x, rl.box[0]);
            dy = min_image(rj.y - ri.y, rl.box[1]);
            dz = (DIM == 3) ? min_image(rj.z - ri.z, rl.box[2]) : 0.0;
            si = ri.sid;
            sj = rj.sid;
            const double bound = rl.R[si] + rl.R[sj] + kWcaCut * (rl.rad[si] + rl.rad[sj]);
            live = dx * dx + dy * dy + dz * dz < bound * bound;
        }
        if (live && tab[si].ne == 0 && tab[sj].ne == 0 && tab[si].nf == 0 && tab[sj].nf == 0) {
            // two points (spheres, disks): the central WCA term of their
            // centres, in FP64, written here; no separation test, no
            // feature stage (no contraction: every kernel variant rounds the
            // term alike)
#pragma clang fp contract(off)
            c_pairs.add(sub1 == 0 ? 1 : 0);
            const double sig = rl.rad[si] + rl.rad[sj], rc = kWcaCut * sig;
            const double r2 = dx * dx + dy * dy + dz * dz;
            c_in.add(sub1 == 0 && r2 < rc * rc ? 1 : 0);
            if (sub1 < 2 && r2 < rc * rc) {  // lane 0 writes i's slot, lane 1 j's
                const double ir2 = 1.0 / r2, s2 = sig * sig * ir2, s6 = s2 * s2 * s2, h = 2.0 * s6 - 1.0;
                const double fr = 24.0 * rl.eps * s6 * h * ir2;  // force on i along x_i - x_j
                const bool js = sub1 == 1;
                const double sg = js ? 1.0 : -1.0;
                SlotRec<T> w;
                w.F[0] = (T)(sg * fr * dx);
                w.F[1] = (T)(sg * fr * dy);
                w.F[2] = (T)(sg * fr * dz);
                w.U = (T)(rl.eps * h * h);
                w.tq[0] = w.tq[1] = w.tq[2] = T(0);
                w.d[0] = (T)(-sg * dx);
                w.d[1] = (T)(-sg * dy);
                w.d[2] = (T)(-sg * dz);
                w.pad1 = T(0);
                set_stamp(w, stamp);
                const int slot = js ? ent.w : ent.z;
                const int pi = js ? ent.y : ent.x;
                if (slot >= 0) {
                    rec[(size_t)slot * N + pi] = w;
                    atomicOr(&l.smask[(size_t)(slot >> 5) * N + pi], 1u << (slot & 31));
                }
            }
            live = false;
        }
        bool need = false;
        if (__ballot(live) != 0) {
            const ShapeTab<T> &Si = tab[si];
            const ShapeTab<T> &Sj = tab[sj];
            M3<T> Rr;
            V3<T> t = v3<T>(0, 0, 0);
            T rc = T(0), Bi = T(0), Bj = T(0);
            for (int k = 0; k < 9; ++k) Rr.m[k] = T(0);
            if (live) {
                Rr = rel_rotation(Ri, Rj);
                t = mulT(Ri, v3<T>((T)dx, (T)dy, (T)dz));
                rc = (T)(kWcaCut * (rl.rad[si] + rl.rad[sj]));
                Bi = (T)rl.R[si] + rc;
                Bj = (T)rl.R[sj] + rc;
            }
            // separation beyond which no feature pair can be inside the
            // cutoff, with room for the rounding of the transformed vertices
            const T thr = rc * T(1.0001) + T(1e-5) * (Bi + Bj);
            V3<T> wj[kVP], wi[kVP];  // this lane's vertices: j's in i's frame, i's in j's frame
            bool hj[kVP], hi[kVP];
#pragma unroll
            for (int p = 0; p < kVP; ++p) {
                const int k = p * kSepLanes + sub1;
                hj[p] = live && k < Sj.nv;
                hi[p] = live && k < Si.nv;
                wj[p] = wi[p] = v3<T>(0, 0, 0);
                if (hj[p]) wj[p] = t + mul(Rr, ld3(Sj.v[k]));
                if (hi[p]) wi[p] = mulT(Rr, ld3(Si.v[k]) - t);
            }
            // bit p of bi (bj): every vertex of j (i) this lane holds lies
            // more than thr beyond supporting plane p of i (j); no early exit
            // and one group reduction at the end, so the plane loads of
            // successive planes overlap
            unsigned bi = 0, bj = 0;
            const int nsi = live ? Si.nsep : 0, nsj = live ? Sj.nsep : 0;
#pragma unroll 2
            for (int p = 0; p < nsi; ++p) {
                const V3<T> n = ld3(Si.sn[p]);
                const T o = Si.so[p];
                bool all = true;
#pragma unroll
                for (int v = 0; v < kVP; ++v) {
                    all &= !hj[v] || dot(n, wj[v]) - o > thr;
                    c_pv.add(hj[v] ? 1 : 0);
                }
                bi |= (all ? 1u : 0u) << p;
            }
#pragma unroll 2
            for (int p = 0; p < nsj; ++p) {
                const V3<T> n = ld3(Sj.sn[p]);
                const T o = Sj.so[p];
                bool all = true;
#pragma unroll
                for (int v = 0; v < kVP; ++v) {
                    all &= !hi[v] || dot(n, wi[v]) - o > thr;
                    c_pv.add(hi[v] ? 1 : 0);
                }
                bj |= (all ? 1u : 0u) << p;
            }
            for (int off = 1; off < kSepLanes; off <<= 1) {
                bi &= __shfl_xor(bi, off, kSepLanes);
                bj &= __shfl_xor(bj, off, kSepLanes);
            }
            const bool sep = (bi | bj) != 0;
            need = live && !sep;
            if (sub1 == 0 && live) {
                c_pairs.add(1);
                c_sep.add(sep ? 1 : 0);
            }
            // queue the pairs that need the feature stage, one entry per group
            const unsigned long long m = __ballot(need && sub1 == 0);
            if constexpr (kSearch) {
                // or, in the split form, append them to the replica's compacted pairs
                if (m != 0) {
                    int at = 0;
                    if (lane == 0) at = atomicAdd(&l.ccount[rl.r], (int)__popcll(m));
                    at = __shfl(at, 0);
                    if (need && sub1 == 0) l.cpairs[rl.poff + at + popc_below(m)] = ent;
                }
            } else if (need && sub1 == 0) {
                QEnt<T> &e = qb[(tail + popc_below(m)) % kQCap];
                e.ent = ent;
                e.si = si;
                e.sj = sj;
                for (int k = 0; k < 9; ++k) {
                    e.Rr[k] = Rr.m[k];
                    e.Ri[k] = Ri.m[k];
                }
                e.t[0] = t.x;
                e.t[1] = t.y;
                e.t[2] = t.z;
                e.d[0] = (T)dx;
                e.d[1] = (T)dy;
                e.d[2] = (T)dz;
            }
            tail += __popcll(m);
        }
        wave_sync_lds();  // the queue entries are visible to every lane
        ++tt;
    }
    if constexpr (kSearch || kForce) {
        // the last workgroup to finish: after the search, the force units
        // of each replica; after the forces, the counts back to zero for
        // the next evaluation (every workgroup has read them by then)
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            rl.last = atomicAdd(&l.ctick[kSearch ? 0 : 1], 1) == (int)gridDim.x - 1 ? 1 : 0;
        }
        __syncthreads();
        if (rl.last) {
            if constexpr (kSearch) {
                const int per_unit = kWaves * (64 / b.pair_lanes);
                for (int q = threadIdx.x; q < b.nrep; q += blockDim.x) {
                    const int c = __hip_atomic_load(&l.ccount[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    l.cunit[q] = (c + per_unit - 1) / per_unit;
                }
                __syncthreads();
                int *part = reinterpret_cast<int *>(pls);  // LDS the search does not use
                const int total = lb::block_scan<64 * kWaves>(l.cunit, l.cunit, b.nrep, part);
                if (threadIdx.x == 0) l.cunit[b.nrep] = total;
            } else {
                for (int q = threadIdx.x; q < b.nrep; q += blockDim.x) l.ccount[q] = 0;
            }
            if (threadIdx.x == 0) l.ctick[kSearch ? 0 : 1] = 0;
        }
    }
    if (COUNT && stats) {
        const unsigned cnt[8] = {c_pairs.get(), c_feat.get(), c_in.get(), c_near.get(), c_ref.get(), c_ee.get(),
                                 c_sep.get(), c_pv.get()};
        const int slot[8] = {ST_PAIRS, ST_FEATURES, ST_INCUT, ST_NEAR, ST_REFINED, ST_EENEAR, ST_SEPARATED, ST_PLANETESTS};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            unsigned long long w = cnt[k];
            for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off, 64);
            if (lane == 0) atomicAdd(&stats[slot[k]], w);
        }
        if (lane == 0 && blockIdx.x == 0 && wid == 0) atomicAdd(&stats[ST_LAUNCHES], 1ull);
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
    if constexpr (NT == 64) {
        // one wavefront: the same pairs as the tree below (lane t adds
        // lane t + off), through lane shuffles instead of LDS and barriers
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        return __shfl(v, 0, 64);
    } else {
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
}

// Nose-Hoover half step of length dt/2 on xi and eta (one variable for
// translation and rotation); returns the velocity scale and updates K.
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

// Per-particle sums of the row-slot records, optionally fused with the
// closing kick.  One block per chunk, so a block belongs to one replica.
// Each particle's row is split over kGatherLanes lanes (lane l takes slots
// l, l + kGatherLanes, ... in order) and combined by a fixed butterfly, so
// the result does not depend on scheduling.  With the kick and NVT each
// block writes its chunk's kinetic partials for k_replica_tail.  A replica
// with no budget left is skipped.
// written row slots a lane loads together in the gather (a record is 48
// bytes in FP32, 96 in FP64; about a quarter of a row's slots are written)
template <typename T>
constexpr int gather_batch() { return 4; }
static_assert(kGatherLanes == 1, "the gather walks a particle's written-slot bits in one lane");

// Adds one row-slot record to a particle's sums: F, tau, U_i = 1/2 sum U_ij
// and W_i = 1/2 sum r_ij (x) F_ij with r_ij = -d.
template <typename T>
__device__ inline void add_slot(double acc[16], const SlotRec<T> &w)
{
    const double f[3] = {(double)w.F[0], (double)w.F[1], (double)w.F[2]};
    for (int a = 0; a < 3; ++a) {
        acc[a] += f[a];
        acc[3 + a] += (double)w.tq[a];
    }
    acc[6] += 0.5 * (double)w.U;
    const double d[3] = {(double)w.d[0], (double)w.d[1], (double)w.d[2]};
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) acc[7 + 3 * a + c] -= 0.5 * d[a] * f[c];
}

// Workgroups of a step's gather beyond its chunk workgroups carry the
// neighbour rows of the step's list build (one wavefront per 4 particles;
// each takes every nrole-th group of the replicas that rebuild), from the
// cells the kick-drift filled.  The pair kernel is done with the rows in
// place; the gather workgroups read records, not rows.
constexpr int kRowWorkgroups = 2048;
inline int row_workgroups(const BatchParams &b) { return pad8(std::min(b.nchunk * (kChunk / lb::kNbrPer), kRowWorkgroups)); }

// The replicas that rebuild are found 64 at a time (one lane each); the
// groups of each are dealt over the role workgroups, starting at a
// replica-dependent workgroup so that small replicas spread out too.
template <int DIM>
__device__ void step_rows(const BatchParams &b, const SysParams *reps, const StatePtrs &s, const ListPtrs &l,
                          const int64_t *budget, int *buf, int first)
{
    const int nrole = (int)gridDim.x - first, me = (int)blockIdx.x - first;
    for (int r0 = 0; r0 < b.nrep; r0 += 64) {
        const int rl = r0 + (int)__lane_id();
        const bool bld = rl < b.nrep && lb::building(LISTS_STEP, rl, reps[rl], l.flags + rl * FLAG_COUNT, budget);
        for (unsigned long long m = __ballot(bld); m != 0ull; m &= m - 1ull) {
            const int r = r0 + __builtin_ctzll(m);
            const SysParams &p = reps[r];
            int32_t *fl = l.flags + r * FLAG_COUNT;
            const int g0 = p.off / lb::kNbrPer, ng = (p.n + lb::kNbrPer - 1) / lb::kNbrPer;
            for (int k = (me + nrole - (int)(((long long)r * 977) % nrole)) % nrole; k < ng; k += nrole)
                lb::nbr_rows<DIM>(b, p, s, l, fl, g0 + k, buf);
        }
    }
}

template <typename T, int DIM, bool KICK>
__global__ void __launch_bounds__(kGatherBlock) k_gather(BatchParams b, const SysParams *reps, StatePtrs s, OutPtrs o,
                                                      ListPtrs l, const SlotRec<T> *__restrict__ rec, double *ke_part,
                                                      double *thermo, int64_t *budget, int64_t *steps)
{
    __shared__ double sh[kGatherBlock];
    const int G = KICK ? pad8(b.nchunk) : (int)gridDim.x;  // chunk workgroups
    if (KICK && (int)blockIdx.x >= G) {
        __shared__ int rbuf[lb::kNbrPer * kRowMax];
        if (l.gflags[G_ANY] != 0) step_rows<DIM>(b, reps, s, l, budget, rbuf, G);
        return;
    }
    constexpr int kB = gather_batch<T>();
    const int sub = threadIdx.x % kGatherLanes;
    const int cb = xcd_block(blockIdx.x, G);  // this block's chunk
    const int i = cb * kGatherPer + threadIdx.x / kGatherLanes;
    if (KICK && blockIdx.x == 0 && threadIdx.x == 0) l.gflags[G_FILL] = l.gflags[G_ANY];  // for the replica tail
    // what depends on the slot alone is requested with the replica's
    // parameters instead of after them (the state only within the length
    // of its arrays).  The records are those of the rows the pair kernel
    // used; a build in this step has already written the next rows, so the
    // written slots are bounded by the row capacity, not the new row length.
    const int nw = slot_words(b.cap);
    uint32_t mw[kRowMax / 32];  // slots written since the last gather, 32 per word
#pragma unroll
    for (int wd = 0; wd < kRowMax / 32; ++wd) mw[wd] = (i < b.N && wd < nw) ? l.smask[(size_t)wd * b.N + i] : 0u;
    double sv[3] = {0.0, 0.0, 0.0}, sL[3] = {0.0, 0.0, 0.0}, sq[4] = {1.0, 0.0, 0.0, 0.0};
    int ssid = 0;
    if (KICK && i < b.nstate) {
        ssid = s.sid[i];
        sv[0] = s.vx[i];
        sv[1] = s.vy[i];
        sL[2] = s.Lz[i];
        if (DIM == 3) {
            sv[2] = s.vz[i];
            sL[0] = s.Lx[i];
            sL[1] = s.Ly[i];
            sq[0] = s.qw[i];
            sq[1] = s.qx[i];
            sq[2] = s.qy[i];
            sq[3] = s.qz[i];
        }
    }
    const unsigned stamp = (unsigned)l.gflags[G_STAMP];  // records of this evaluation only
    const int r = cb < b.nchunk ? l.chunk_rep[cb] : -1;
    if (r < 0) return;
    const SysParams &p = reps[r];
    if (KICK && threadIdx.x == 0 && cb == p.off / kChunk) {
        // whether the replica tail writes this step's new pair entries (the
        // tail itself moves the rebuild flag on)
        int32_t *fl = l.flags + r * FLAG_COUNT;
        fl[FLAG_FILL] = (fl[FLAG_REBUILD] != 0 && budget[r] > 0) ? 1 : 0;
    }
    if (KICK && budget[r] <= 0) return;
    const bool npt = KICK && p.ensemble == DEM_NPT;
    const bool nvt = KICK && (p.ensemble == DEM_NVT || npt);
    const size_t N = (size_t)b.N;
    const bool mine = i < p.off + p.n;
    double acc[16];
    for (int c = 0; c < 16; ++c) acc[c] = 0.0;  // F[3], T[3], U, W[9]
    if (mine) {
        // only the slots written since the last gather, whose words are
        // cleared for the next evaluation; ascending, so they are added in
        // row order.  Loads go in batches: every load of a batch is issued
        // before any of its sums, so the batch's round trips overlap.
#pragma unroll
        for (int wd = 0; wd < kRowMax / 32; ++wd) {
            uint32_t bits = mw[wd];
            if (bits == 0u) continue;
            l.smask[(size_t)wd * N + i] = 0u;
            while (bits != 0u) {
                SlotRec<T> w[kB];
                bool h[kB];
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    h[u] = bits != 0u;
                    const int k = 32 * wd + (h[u] ? __builtin_ctz(bits) : 0);
                    w[u] = h[u] ? rec[(size_t)k * N + i] : SlotRec<T>{};
                    bits &= bits - 1u;
                }
                __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the sums
#pragma unroll
                for (int u = 0; u < kB; ++u)
                    if (h[u] && slot_stamp(w[u]) == stamp) add_slot(acc, w[u]);
            }
        }
    }
    for (int off = 1; off < kGatherLanes; off <<= 1)
        for (int c = 0; c < 16; ++c) acc[c] += __shfl_xor(acc[c], off, kGatherLanes);
    double kt = 0.0, kr = 0.0, tw = 0.0;
    if (mine && sub == 0) {
        double *F = acc, *Tq = acc + 3;
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
        o.U[i] = acc[6];
        for (int c = 0; c < 9; ++c) o.W[(size_t)c * b.wstride + i] = acc[7 + c];
        if (KICK) {
            const int sid = ssid;
            const double hm = 0.5 * p.dt / p.mass[sid];
            double v[3] = {sv[0] + hm * F[0], sv[1] + hm * F[1], 0.0};
            if (npt) {  // the kick's exact flow with the barostat's friction
                const double *th = thermo + r * TH_COUNT;
                const double damp = th[TH_DAMP], fk = th[TH_FK] / p.mass[sid];
                for (int a = 0; a < DIM; ++a) v[a] = sv[a] * damp + fk * F[a];
            }
            s.vx[i] = v[0];
            s.vy[i] = v[1];
            double L[3] = {0.0, 0.0, 0.0};
            if (DIM == 3) {
                if (!npt) v[2] = sv[2] + hm * F[2];
                s.vz[i] = v[2];
                double tb[3];
                body_torque(sq, Tq[0], Tq[1], Tq[2], tb);
                L[0] = sL[0] + 0.5 * p.dt * tb[0];
                L[1] = sL[1] + 0.5 * p.dt * tb[1];
                L[2] = sL[2] + 0.5 * p.dt * tb[2];
                s.Lx[i] = L[0];
                s.Ly[i] = L[1];
                s.Lz[i] = L[2];
            } else {
                L[2] = sL[2] + 0.5 * p.dt * Tq[2];
                s.Lz[i] = L[2];
            }
            if (nvt) {
                kt = 0.5 * p.mass[sid] * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                for (int a = 0; a < 3; ++a)
                    if (p.inertia[sid][a] > 0.0) kr += 0.5 * L[a] * L[a] / p.inertia[sid][a];
            }
            if (npt) tw = acc[7] + acc[11] + (DIM == 3 ? acc[15] : 0.0);
        }
    }
    if (!nvt) return;
    kt = block_sum<kGatherBlock>(kt, sh);
    kr = block_sum<kGatherBlock>(kr, sh);
    if (npt) tw = block_sum<kGatherBlock>(tw, sh);
    if (threadIdx.x == 0) {
        ke_part[kKePer * cb] = kt;
        ke_part[kKePer * cb + 1] = kr;
        ke_part[kKePer * cb + 2] = tw;
    }
}

// The end of a step for each replica (one block per replica slot, after
// k_gather): the thermostat's closing half step and the next step's
// opening half step from the kinetic energy after the closing kick (the
// gather's partial sums per chunk, added in chunk order), the step budget
// and count, and the list-rebuild transitions: this step's build is
// counted, and a trigger raised during the step schedules a build for the
// next step.  A kernel of its own, so the partial sums are visible without
// a device-wide fence in every gather block.  Workgroups beyond the
// replica slots carry the end of the step's list build: the tile plan (the
// first of them) and the pair entries of every chunk of a replica that
// rebuilds (FLAG_FILL, which the tail workgroups do not touch), one chunk
// per workgroup at a time; the cells are emptied for the next build.
__global__ void __launch_bounds__(kGatherBlock) k_replica_tail(BatchParams b, SysParams *reps, ListPtrs l,
                                                               const double *ke_part, double *thermo, int64_t *budget,
                                                               int64_t *steps)
{
    __shared__ double sh[kGatherBlock];
    if ((int)blockIdx.x >= b.nrep) {
        static_assert(kGatherBlock == kChunk, "one wavefront per chunk");
        __shared__ int part[kGatherBlock];
        if (l.gflags[G_FILL] == 0) return;
        const int fb = (int)blockIdx.x - b.nrep, nfb = (int)gridDim.x - b.nrep;
        if (fb == 0)
            lb::plan<kGatherBlock>(b, reps, l, part, [&](int r) {
                return reps[r].n > 0 && l.flags[r * FLAG_COUNT + FLAG_FILL] != 0;
            });
        // the replicas that rebuild, 64 at a time; their chunks dealt over
        // the fill workgroups from a replica-dependent start
        for (int r0 = 0; r0 < b.nrep; r0 += 64) {
            const int rl = r0 + (int)__lane_id();
            const bool bld = rl < b.nrep && reps[rl].live && reps[rl].n > 0 && l.flags[rl * FLAG_COUNT + FLAG_FILL] != 0;
            for (unsigned long long m = __ballot(bld); m != 0ull; m &= m - 1ull) {
                const int r = r0 + __builtin_ctzll(m);
                const SysParams &p = reps[r];
                const int c0 = p.off / kChunk, nc = (p.n + kChunk - 1) / kChunk;
                for (int k = (fb + nfb - (int)(((long long)r * 977) % nfb)) % nfb; k < nc; k += nfb)
                    lb::fill_chunk(b, p, l, c0 + k, false, true);
            }
        }
        return;
    }
    const int r = blockIdx.x;
    int32_t *fl = l.flags + r * FLAG_COUNT;
    double *th = thermo + r * TH_COUNT;
    // the slot's step values are requested together with its parameters
    // (the thermostat slots exist for every replica slot)
    const int64_t left = budget[r];
    const int32_t rebuilt = fl[FLAG_REBUILD], trigger = fl[FLAG_TRIGGER];
    const double xi0 = th[TH_XI], eta0 = th[TH_ETA];
    SysParams &p = reps[r];
    if (!p.live || p.n == 0 || left <= 0) return;
    if (p.ensemble == DEM_NPT) {
        // closing of this step: barostat half step (K_trans after the
        // closing kick, the virial of this step's forces, this step's box),
        // thermostat half step; opening of the next: thermostat, barostat;
        // then the next step's kick and drift factors and its box
        const int nblk = (p.n + kChunk - 1) / kChunk;
        const int c0 = p.off / kChunk;
        double at = 0.0, ar = 0.0, aw = 0.0;
#pragma unroll 8
        for (int c = threadIdx.x; c < nblk; c += blockDim.x) {
            at += ke_part[kKePer * (c0 + c)];
            ar += ke_part[kKePer * (c0 + c) + 1];
            aw += ke_part[kKePer * (c0 + c) + 2];
        }
        double Kt2 = 2.0 * block_sum<kGatherBlock>(at, sh);
        const double Kr2 = 2.0 * block_sum<kGatherBlock>(ar, sh);
        const double trW = block_sum<kGatherBlock>(aw, sh);
        if (threadIdx.x == 0) {
            double xi = xi0, eta = eta0, veps = th[TH_VEPS];
            baro_half(p, Kt2, trW, veps);
            double K2 = Kt2 + Kr2;
            const double sb = nh_half_npt(p, xi, eta, K2, veps);
            Kt2 *= sb * sb;
            th[TH_XI_B] = xi;
            th[TH_ETA_B] = eta;
            th[TH_VEPS_B] = veps;
            th[TH_SB] = sb;
            const double sa = nh_half_npt(p, xi, eta, K2, veps);
            Kt2 *= sa * sa;
            baro_half(p, Kt2, trW, veps);
            th[TH_XI] = xi;
            th[TH_ETA] = eta;
            th[TH_VEPS] = veps;
            th[TH_SA] = sa;
            th[TH_OPEN] = 1.0;
            npt_factors(p, veps, th);
            if (rebuilt != 0)  // this step's lists were built in this step's box
                for (int a = 0; a < 3; ++a) p.box_build[a] = p.box[a];
            double box[3];
            for (int a = 0; a < 3; ++a) {
                th[TH_BOXN + a] = p.box[a];
                box[a] = p.box[a] * th[TH_GROW];
            }
            set_box(p, box, fl);
        }
    }
    if (p.ensemble == DEM_NVT) {
        const int nblk = (p.n + kChunk - 1) / kChunk;
        const int c0 = p.off / kChunk;
        double acc2 = 0.0;
        // unrolled so that many loads are in flight at once (large
        // replicas have thousands of chunks); the sums keep their order
#pragma unroll 8
        for (int c = threadIdx.x; c < nblk; c += blockDim.x)
            acc2 += ke_part[kKePer * (c0 + c)] + ke_part[kKePer * (c0 + c) + 1];
        double K = block_sum<kGatherBlock>(acc2, sh);
        if (threadIdx.x == 0) {
            double xi = xi0, eta = eta0;
            const double sb = nh_half(p, xi, eta, K);  // closes this step
            th[TH_XI_B] = xi;
            th[TH_ETA_B] = eta;
            th[TH_SB] = sb;
            const double sa = nh_half(p, xi, eta, K);  // opens the next step
            th[TH_XI] = xi;
            th[TH_ETA] = eta;
            th[TH_SA] = sa;
            th[TH_OPEN] = 1.0;
        }
    }
    if (threadIdx.x == 0) {
        budget[r] = left - 1;
        steps[r] += 1;
        if (rebuilt != 0) {  // this step's lists are built: count them
            fl[FLAG_REBUILD] = 0;
            fl[FLAG_NBUILDS] += 1;
            atomicSub(&l.gflags[G_ANY], 1);
        }
        if (trigger != 0) {  // the next step rebuilds
            fl[FLAG_TRIGGER] = 0;
            fl[FLAG_REBUILD] = 1;
            atomicAdd(&l.gflags[G_ANY], 1);
        }
    }
}

template <typename T>
__global__ void k_rotations(BatchParams b, const SysParams *reps, StatePtrs s, ListPtrs l, PartRec<T> *rot,
                            PartRec64 *rec64)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = i / kChunk;
    if (c >= b.nchunk) return;
    const int r = l.chunk_rep[c];
    if (r < 0 || i >= reps[r].off + reps[r].n) return;
    double R[9];
    quat_to_rot(s.qw[i], s.qx[i], s.qy[i], s.qz[i], R);
    PartRec<T> rc;
    rc.x = s.x[i];
    rc.y = s.y[i];
    rc.z = b.dim == 3 ? s.z[i] : 0.0;
    for (int k = 0; k < 9; ++k) rc.R[k] = (T)R[k];
    rc.sid = s.sid[i];
    rot[i] = rc;
    if (sizeof(T) == 4) rec64[i] = PartRec64{rc.x, rc.y, rc.z, s.qw[i], s.qx[i], s.qy[i], s.qz[i], 0.0};
}

template <typename T, int DIM, int GL, int OCC, int SL, int STAGE, bool FC>
void pairs_t(const Launch &L, unsigned long long *stats, hipStream_t stream);

// The compiled shapes: {8, 16} lanes per pair x {2, 3} wavefronts per SIMD
// with the 4-lane separation stage, and 16 lanes x {2, 3} with the 16-lane
// one; in the split form, the search kernel (4-lane separation stage,
// kSearchOcc wavefronts per SIMD) and then the force kernel at {8, 16}
// lanes x {2, 3} wavefronts.  Each feature stage with the supporting-plane
// prefilter or with the shape-local feature cells (FC); the FC feature
// stage does not fit the 168 registers of 3 wavefronts per SIMD, so it is
// compiled for 2 whatever the shape asks.
template <typename T, int DIM, bool FC>
void pairs_form(const Launch &L, unsigned long long *stats, hipStream_t stream)
{
    const bool g8 = L.b.pair_lanes == 8, o3 = !FC && L.b.pair_waves == 3;
    constexpr int O3 = FC ? 2 : 3;  // (FC: never taken, o3 is false)
    if (L.b.pair_split) {
        pairs_t<T, DIM, 16, kSearchOcc, 4, kSearchOnly, false>(L, stats, stream);
        if (g8)
            o3 ? pairs_t<T, DIM, 8, O3, 4, kForces, FC>(L, stats, stream) : pairs_t<T, DIM, 8, 2, 4, kForces, FC>(L, stats, stream);
        else
            o3 ? pairs_t<T, DIM, 16, O3, 4, kForces, FC>(L, stats, stream)
               : pairs_t<T, DIM, 16, 2, 4, kForces, FC>(L, stats, stream);
    } else if (L.b.pair_sep == 16)
        o3 ? pairs_t<T, DIM, 16, O3, 16, kFused, FC>(L, stats, stream) : pairs_t<T, DIM, 16, 2, 16, kFused, FC>(L, stats, stream);
    else if (g8)
        o3 ? pairs_t<T, DIM, 8, O3, 4, kFused, FC>(L, stats, stream) : pairs_t<T, DIM, 8, 2, 4, kFused, FC>(L, stats, stream);
    else
        o3 ? pairs_t<T, DIM, 16, O3, 4, kFused, FC>(L, stats, stream) : pairs_t<T, DIM, 16, 2, 4, kFused, FC>(L, stats, stream);
}

template <typename T, int DIM>
void pairs_shape(const Launch &L, unsigned long long *stats, hipStream_t stream)
{
    if (L.b.feature_cells) pairs_form<T, DIM, true>(L, stats, stream);
    else pairs_form<T, DIM, false>(L, stats, stream);
}

template <typename T, int DIM, int GL, int OCC, int SL, int STAGE, bool FC>
void pairs_t(const Launch &L, unsigned long long *stats, hipStream_t stream)
{
    const size_t sh = pair_kernel_lds(sizeof(T) == 4 ? DEM_FP32 : DEM_FP64, L.b.tab_slots, GL, SL, STAGE, FC ? 1 : 0);
    const int grid = STAGE == kSearchOnly ? L.b.search_blocks : L.b.pair_blocks;
    const auto rot = reinterpret_cast<const PartRec<T> *>(L.f.rot);
    const auto rec = reinterpret_cast<SlotRec<T> *>(L.f.rec);
    const auto tab = reinterpret_cast<const ShapeTab<T> *>(L.f.tab);
    const auto tab64 = reinterpret_cast<const ShapeTab<double> *>(L.f.tab64);
    if (stats)
        k_pairs<T, DIM, GL, true, OCC, SL, STAGE, FC><<<grid, 64 * kWaves, sh, stream>>>(L.b, L.reps, L.s, L.l, rot,
                                                                                      L.f.rec64, rec, tab, tab64, stats);
    else
        k_pairs<T, DIM, GL, false, OCC, SL, STAGE, FC><<<grid, 64 * kWaves, sh, stream>>>(L.b, L.reps, L.s, L.l, rot,
                                                                                       L.f.rec64, rec, tab, tab64, nullptr);
}

template <typename T, int DIM>
void gather_t(const Launch &L, bool kick, hipStream_t stream)
{
    const SlotRec<T> *rec = reinterpret_cast<const SlotRec<T> *>(L.f.rec);
    if (kick) {
        k_gather<T, DIM, true><<<pad8(L.b.nchunk) + row_workgroups(L.b), kGatherBlock, 0, stream>>>(
            L.b, L.reps, L.s, L.o, L.l, rec, L.ke_part, L.thermo, L.budget, L.steps);
        k_replica_tail<<<L.b.nrep + std::min(L.b.nchunk, 1024), kGatherBlock, 0, stream>>>(
            L.b, const_cast<SysParams *>(L.reps), L.l, L.ke_part, L.thermo, L.budget, L.steps);
    }
    else
        k_gather<T, DIM, false><<<pad8(L.b.nchunk), kGatherBlock, 0, stream>>>(L.b, L.reps, L.s, L.o, L.l, rec, L.ke_part,
                                                                     L.thermo, L.budget, L.steps);
}

}  // namespace

void launch_rotations(const Launch &L, hipStream_t stream)
{
    if (L.b.nchunk == 0) return;
    const int nb = blocks_for(L.b.nchunk * kChunk);
    if (L.precision == DEM_FP32)
        k_rotations<float><<<nb, kBlock, 0, stream>>>(L.b, L.reps, L.s, L.l, reinterpret_cast<PartRec<float> *>(L.f.rot),
                                                      L.f.rec64);
    else
        k_rotations<double><<<nb, kBlock, 0, stream>>>(L.b, L.reps, L.s, L.l, reinterpret_cast<PartRec<double> *>(L.f.rot),
                                                       L.f.rec64);
}

void launch_pairs(const Launch &L, unsigned long long *stats, hipStream_t stream)
{
    if (L.b.nchunk == 0) return;
    if (L.precision == DEM_FP32) {
        if (L.b.dim == 3) pairs_shape<float, 3>(L, stats, stream);
        else pairs_shape<float, 2>(L, stats, stream);
    } else {
        if (L.b.dim == 3) pairs_shape<double, 3>(L, stats, stream);
        else pairs_shape<double, 2>(L, stats, stream);
    }
}

void launch_gather(const Launch &L, bool kick, hipStream_t stream)
{
    if (L.b.nchunk == 0) return;
    if (L.precision == DEM_FP32) {
        if (L.b.dim == 3) gather_t<float, 3>(L, kick, stream);
        else gather_t<float, 2>(L, kick, stream);
    } else {
        if (L.b.dim == 3) gather_t<double, 3>(L, kick, stream);
        else gather_t<double, 2>(L, kick, stream);
    }
}

size_t pair_kernel_lds(int precision, int tab_slots, int lanes, int sep, int stage, int fc)
{
    const size_t w = precision == DEM_FP32 ? sizeof(ShapeTab<float>) : sizeof(ShapeTab<double>);
    const size_t pl = precision == DEM_FP32 ? sizeof(PairLds<float>) : sizeof(PairLds<double>);
    const size_t qe = precision == DEM_FP32 ? sizeof(QEnt<float>) : sizeof(QEnt<double>);
    const size_t acc = precision == DEM_FP32 ? sizeof(Acc<float>) : sizeof(Acc<double>);
    if (stage == kSearchOnly)  // tables, replica, and the last workgroup's scan
        return (size_t)tab_slots * w + sizeof(RepLds) + sizeof(int) * 64 * kWaves;
    return (size_t)tab_slots * w + sizeof(RepLds) + kWaves * (64 / lanes) * pl + kWaves * queue_slots(sep, lanes) * qe +
           (lanes == 16 ? kWaves * 64 * acc : 0) + (fc ? kWaves * (64 / lanes) * sizeof(PairFc) : 0);
}

namespace {
template <typename T, int DIM, int STAGE, bool FC>
hipError_t pair_occupancy(int *per_cu, size_t lds, int lanes, int waves, int sep)
{
    const int t = 64 * kWaves;
    auto occ = [&](auto kernel) { return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kernel, t, lds); };
    constexpr int O3 = FC ? 2 : 3;  // the FC feature stage is compiled for 2 wavefronts per SIMD only
    if constexpr (STAGE == kSearchOnly) {
        return occ(k_pairs<T, DIM, 16, false, kSearchOcc, 4, kSearchOnly, false>);
    } else {
        if constexpr (STAGE == kFused)
            if (sep == 16)
                return waves == 3 ? occ(k_pairs<T, DIM, 16, false, O3, 16, STAGE, FC>)
                                  : occ(k_pairs<T, DIM, 16, false, 2, 16, STAGE, FC>);
        if (lanes == 8)
            return waves == 3 ? occ(k_pairs<T, DIM, 8, false, O3, 4, STAGE, FC>) : occ(k_pairs<T, DIM, 8, false, 2, 4, STAGE, FC>);
        return waves == 3 ? occ(k_pairs<T, DIM, 16, false, O3, 4, STAGE, FC>) : occ(k_pairs<T, DIM, 16, false, 2, 4, STAGE, FC>);
    }
}

template <typename T, int DIM>
hipError_t pair_occupancy_stage(int *per_cu, size_t lds, int lanes, int waves, int sep, int stage, int fc)
{
    if (stage == kSearchOnly) return pair_occupancy<T, DIM, kSearchOnly, false>(per_cu, lds, lanes, waves, sep);
    if (stage == kForces)
        return fc ? pair_occupancy<T, DIM, kForces, true>(per_cu, lds, lanes, waves, sep)
                  : pair_occupancy<T, DIM, kForces, false>(per_cu, lds, lanes, waves, sep);
    return fc ? pair_occupancy<T, DIM, kFused, true>(per_cu, lds, lanes, waves, sep)
              : pair_occupancy<T, DIM, kFused, false>(per_cu, lds, lanes, waves, sep);
}
}  // namespace

int pair_blocks_resident(int precision, int dim, int tab_slots, int lanes, int waves, int sep, int stage, int fc)
{
    const size_t lds = pair_kernel_lds(precision, tab_slots, lanes, sep, stage, fc);
    int per_cu = 0, cus = 0, dev = 0;
    hipError_t e;
    if (precision == DEM_FP32)
        e = dim == 3 ? pair_occupancy_stage<float, 3>(&per_cu, lds, lanes, waves, sep, stage, fc)
                     : pair_occupancy_stage<float, 2>(&per_cu, lds, lanes, waves, sep, stage, fc);
    else
        e = dim == 3 ? pair_occupancy_stage<double, 3>(&per_cu, lds, lanes, waves, sep, stage, fc)
                     : pair_occupancy_stage<double, 2>(&per_cu, lds, lanes, waves, sep, stage, fc);
    if (e != hipSuccess || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 512;
    return std::max(8, per_cu * cus);
}

}  // namespace dem

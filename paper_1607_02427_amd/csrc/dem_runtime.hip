// libdem host runtime: the C ABI of dem.h.
//
// A handle is a batch of replicas (a single system is a batch of one).  It
// owns the device copies of the shape tables (FP64 and FP32), the replica
// parameter table, the cell and neighbour lists of every replica, flags,
// reduction scratch and one captured graph of a whole time step, which
// dem_step replays for every live replica at once.  A single system uses
// the caller's state and output arrays in place; a batch keeps its
// replicas' state in arrays of its own (particle slots, 64 to a chunk,
// handed out first-fit) and copies it in and out on request.  Every launch
// goes to the handle's stream; graphs are recorded on a private stream and
// launched on the handle's.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "dem_internal.h"

using namespace dem;

namespace {

// First-fit allocator over slots [0, size).
struct SlotArena {
    std::vector<uint8_t> used;
    void reset(int size) { used.assign((size_t)std::max(size, 0), 0); }
    int size() const { return (int)used.size(); }
    // first offset of `count` free slots, or -1
    int find(int count) const
    {
        if (count == 0) return 0;
        int run = 0;
        for (int k = 0; k < size(); ++k) {
            run = used[k] ? 0 : run + 1;
            if (run == count) return k - count + 1;
        }
        return -1;
    }
    void mark(int off, int count, uint8_t v)
    {
        for (int k = off; k < off + count; ++k) used[k] = v;
    }
    // one past the last used slot
    int high() const
    {
        for (int k = size(); k > 0; --k)
            if (used[k - 1]) return k;
        return 0;
    }
    int free_slots() const
    {
        int f = 0;
        for (uint8_t u : used) f += u ? 0 : 1;
        return f;
    }
};

struct Replica {
    bool live = false;
    bool on_device = false;      // its SysParams have been uploaded (the device's box is current)
    size_t bytes = 0;            // device bytes charged against the batch's admission budget
    SysParams sp{};
    dem_params prm{};            // copy; shapes not kept
    double r_list = 0.0;
    int chunk0 = 0, nchunks = 0;
    int cell0 = 0, ncells = 0;
    int shape0 = 0, nshapes = 0;
};

}  // namespace

struct dem_system {
    bool batch = false;
    size_t hbm_budget = 0, hbm_used = 0;  // admission budget (0: none) and the live replicas' charge
    int dim = 0, precision = 0;
    bool auto_cap = true;
    bool counting = false;
    int pair_lanes = kDefaultPairLanes;  // pair-kernel shape: lanes per pair,
    int pair_grid = 1;                   // blocks per resident block slot
    int pair_waves = kDefaultPairWaves;  // wavefronts per SIMD
    int pair_sep = kDefaultPairSep;      // and lanes per pair of its separation stage;
    int pair_split = 0;                  // 1: search and force kernels instead of one
    int feature_cells = 0;               // 1: the feature search reads the shape-local cells
    BatchParams bp{};
    std::vector<Replica> reps;
    SlotArena chunks, cells, shapes;
    int Ncap = 0;                // particle slots
    SysParams *d_reps = nullptr;
    int32_t *d_chunk_rep = nullptr;
    std::vector<int32_t> h_chunk_rep;
    StatePtrs st{};
    OutPtrs out{};
    ListPtrs lst{};
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    void *tab64 = nullptr, *tab32 = nullptr;
    uint2 *fcells = nullptr;             // [shape slots][kFcCells] shape-local feature cells
    void *rot = nullptr;         // [N] PartRec in the force precision
    PartRec64 *rec64 = nullptr;  // [N] FP64 position and orientation (FP32 path)
    void *rec = nullptr;         // [cap][N] SlotRec in the force precision
    double *ke_part = nullptr;   // [kKePer * chunks]
    double *e_part = nullptr;    // [12 * chunks]
    double *scratch = nullptr;   // this device's copy of the static energy scratch (device address)
    double *thermo = nullptr;    // [replica][TH_COUNT]
    int64_t *budget = nullptr;   // [replica] steps left
    int64_t *steps = nullptr;    // [replica] steps done
    unsigned long long *stats = nullptr;
    hipGraph_t graph = nullptr, graph_multi = nullptr;  // one step; kGraphSteps steps
    hipGraphExec_t gexec = nullptr, gexec_multi = nullptr;
    std::string err;
};

namespace {

std::string g_err;
constexpr int64_t kUnbounded = (int64_t)1 << 62;


dem_status fail(dem_system *h, dem_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    g_err = buf;
    return s;
}

// Device memory of dem_replica_energy_noalloc, which allocates nothing: the
// per-chunk partials of one replica (12 doubles per 64-particle chunk, at
// most kScratchChunks chunks) and their 12 totals.  Each device holds its
// own copy until the process ends; in host code `scratch` names no device
// address, so host code uses only the address that hipGetSymbolAddress
// returns for the current device (scratch_of).
constexpr int kScratchChunks = 4096;  // replicas of up to 262,144 particles
constexpr size_t kScratchTotals = (size_t)12 * kScratchChunks;
__device__ __align__(256) double scratch[kScratchTotals + 16];

constexpr int kMaxDevices = 64;
double *g_scratch_addr[kMaxDevices];
std::mutex g_scratch_mu;

// The current device's address of `scratch`, looked up once per device at
// handle creation (with that device current).
dem_status scratch_of(dem_system *h)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(h, DEM_E_HIP, "no current device for the static scratch");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(h, DEM_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_addr[dev] = static_cast<double *>(ptr);
    }
    h->scratch = g_scratch_addr[dev];
    return DEM_OK;
}

#define HIPCHK(h, call)                                                                            \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return fail(h, DEM_E_HIP, "%s: %s", #call, hipGetErrorString(e_));  \
    } while (0)

__global__ void k_set_i32(int32_t *p, int32_t v) { *p = v; }
__global__ void k_bump(int32_t *p) { *p += 1; }
__global__ void k_set_i64(int64_t *p, int64_t v) { *p = v; }
// A replica without particles advances by bookkeeping only.
__global__ void k_advance_empty(int64_t *budget, int64_t *steps, int64_t n)
{
    const int64_t d = *budget < n ? *budget : n;
    if (d > 0) {
        *budget -= d;
        *steps += d;
    }
}
__global__ void k_count_build(int32_t *flags) { flags[FLAG_NBUILDS] += 1; }
// A replica leaves the batch: drop its pending list build from the count.
__global__ void k_retire_flags(int32_t *flags, int32_t *gflags)
{
    if (flags[FLAG_REBUILD] != 0) atomicSub(&gflags[G_ANY], 1);
    for (int w = 0; w < FLAG_COUNT; ++w) flags[w] = 0;
}
__global__ void k_set_thermo(double *th, double xi, double eta)
{
    th[TH_XI] = th[TH_XI_B] = xi;
    th[TH_ETA] = th[TH_ETA_B] = eta;
    th[TH_SB] = th[TH_SA] = 1.0;
    th[TH_OPEN] = 0.0;
}

// A new replica's barostat words (v_eps = 0) and the box of its positions.
__global__ void k_set_baro(double *th, double bx, double by, double bz)
{
    th[TH_VEPS] = th[TH_VEPS_B] = 0.0;
    th[TH_DAMP] = th[TH_GROW] = 1.0;
    th[TH_FK] = th[TH_VFAC] = 0.0;
    th[TH_BOXN] = bx;
    th[TH_BOXN + 1] = by;
    th[TH_BOXN + 2] = bz;
}

// The barostat velocity; the next step opens from it.
__global__ void k_set_veps(double *th, double veps)
{
    th[TH_VEPS] = th[TH_VEPS_B] = veps;
    th[TH_XI] = th[TH_XI_B];
    th[TH_ETA] = th[TH_ETA_B];
    th[TH_SB] = th[TH_SA] = 1.0;
    th[TH_OPEN] = 0.0;
}

// Lists just built from the current positions: an NPT replica's build box.
__global__ void k_box_built(SysParams *reps, int r)
{
    for (int a = 0; a < 3; ++a) reps[r].box_build[a] = reps[r].box[a];
}

// An NPT replica's box (and cells) from the box of its positions in its
// thermostat words, after those were restored from a checkpoint.
__global__ void k_box_restore(SysParams *reps, int r, ListPtrs l, const double *thermo)
{
    SysParams &p = reps[r];
    if (p.ensemble != DEM_NPT) return;
    set_box(p, thermo + r * TH_COUNT + TH_BOXN, l.flags + r * FLAG_COUNT);
    for (int a = 0; a < 3; ++a) p.box_build[a] = p.box[a];
}

struct HostVec {
    double x, y, z;
};
inline HostVec hsub(HostVec a, HostVec b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline HostVec hcross(HostVec a, HostVec b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double hdot(HostVec a, HostVec b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// Supporting planes of the inner body (the vertices' convex hull lies on
// their inner side): in 3D every face plane that has no vertex beyond it
// (all of them for a convex body), in 2D every edge line with all vertices
// on one side, its normal pointing away from them.  The offset is the exact
// support value max_k n.v_k, so a point farther than r_cut beyond such a
// plane is farther than r_cut from every feature of the body.
void support_planes(ShapeTab<double> &T, int dim)
{
    T.nsep = 0;
    const double tol = 1e-9 * (1.0 + T.R);
    auto support = [&](HostVec n) {
        double hi = -1e300;
        for (int k = 0; k < T.nv; ++k) hi = std::max(hi, hdot(n, HostVec{T.v[k][0], T.v[k][1], T.v[k][2]}));
        return hi;
    };
    auto add = [&](HostVec n, double o) {
        if (T.nsep >= kMaxSep) return;
        T.sn[T.nsep][0] = n.x;
        T.sn[T.nsep][1] = n.y;
        T.sn[T.nsep][2] = n.z;
        T.so[T.nsep] = o;
        ++T.nsep;
    };
    if (dim == 3) {
        for (int f = 0; f < T.nf; ++f) {
            const HostVec n{T.fn[f][0], T.fn[f][1], T.fn[f][2]};
            const double hi = support(n);
            if (hi <= T.fo[f] + tol) add(n, hi);
        }
    } else {
        for (int k = 0; k < T.ne; ++k) {
            const double l = std::sqrt(T.el2[k]);
            const HostVec n{T.ed[k][1] / l, -T.ed[k][0] / l, 0.0};
            const HostVec a{T.v[T.e[k][0]][0], T.v[T.e[k][0]][1], 0.0};
            const double o = hdot(n, a);
            const double hi = support(n), lo = -support(HostVec{-n.x, -n.y, 0.0});
            if (hi <= o + tol) add(n, hi);
            else if (lo >= o - tol) add(HostVec{-n.x, -n.y, 0.0}, -lo);
        }
    }
}

// Validates one shape and fills the FP64 table.
dem_status build_table(dem_system *h, int idx, const dem_shape_desc &d, int dim, ShapeTab<double> &T)
{
    std::memset(&T, 0, sizeof T);
    if (d.dim != dim) return fail(h, DEM_E_SHAPE, "shape %d: dim %d differs from system dim %d", idx, d.dim, dim);
    // a single point (no edges, no faces) is a sphere or disk of the rounding radius
    const bool point = d.n_vertices == 1 && d.n_edges == 0 && (dim == 2 || d.n_faces == 0);
    if (!point) {
        if (d.n_vertices < (dim == 3 ? 4 : 3) || d.n_vertices > DEM_MAX_VERTS)
            return fail(h, DEM_E_SHAPE, "shape %d: %d vertices (limit %d)", idx, d.n_vertices, DEM_MAX_VERTS);
        if (d.n_edges < 3 || d.n_edges > DEM_MAX_EDGES)
            return fail(h, DEM_E_SHAPE, "shape %d: %d edges (limit %d)", idx, d.n_edges, DEM_MAX_EDGES);
        if (dim == 3 && (d.n_faces < 4 || d.n_faces > DEM_MAX_FACES))
            return fail(h, DEM_E_SHAPE, "shape %d: %d faces (limit %d)", idx, d.n_faces, DEM_MAX_FACES);
    }
    if (!d.vertices || (!point && (!d.edges || (dim == 3 && (!d.face_offsets || !d.face_vertices)))))
        return fail(h, DEM_E_SHAPE, "shape %d: null table", idx);
    if (!(d.rounding_radius > 0.0) || !(d.mass > 0.0))
        return fail(h, DEM_E_SHAPE, "shape %d: rounding radius and mass must be positive", idx);
    for (int a = (dim == 3 ? 0 : 2); a < 3; ++a)
        if (!(d.inertia[a] > 0.0)) return fail(h, DEM_E_SHAPE, "shape %d: principal moment %d must be positive", idx, a);
    T.nv = d.n_vertices;
    T.ne = d.n_edges;
    T.nf = dim == 3 ? d.n_faces : 0;
    T.r = d.rounding_radius;
    double R = 0.0;
    for (int k = 0; k < T.nv; ++k) {
        for (int a = 0; a < 3; ++a) T.v[k][a] = d.vertices[3 * k + a];
        if (dim == 2 && T.v[k][2] != 0.0) return fail(h, DEM_E_SHAPE, "shape %d: 2D vertex %d has z != 0", idx, k);
        const double *v = d.vertices + 3 * k;
        double rr = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (rr > R) R = rr;
    }
    T.R = R;
    if (point && R != 0.0) return fail(h, DEM_E_SHAPE, "shape %d: a point shape's vertex must be its centre", idx);
    for (int k = 0; k < T.ne; ++k) {
        int a = d.edges[2 * k], b = d.edges[2 * k + 1];
        if (a < 0 || b < 0 || a >= T.nv || b >= T.nv || a == b)
            return fail(h, DEM_E_SHAPE, "shape %d: bad edge %d (%d, %d)", idx, k, a, b);
        T.e[k][0] = a;
        T.e[k][1] = b;
        double l2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            T.ed[k][c] = T.v[b][c] - T.v[a][c];
            l2 += T.ed[k][c] * T.ed[k][c];
        }
        if (!(l2 > 0.0)) return fail(h, DEM_E_SHAPE, "shape %d: edge %d has zero length", idx, k);
        T.el2[k] = l2;
        T.einv[k] = 1.0 / l2;
        T.eh[k] = 0.5 * std::sqrt(l2);
        for (int c = 0; c < 3; ++c) T.em[k][c] = 0.5 * (T.v[a][c] + T.v[b][c]);
    }
    if (dim == 3 && !point) {
        if (d.face_offsets[0] != 0) return fail(h, DEM_E_SHAPE, "shape %d: face_offsets[0] != 0", idx);
        if (d.face_offsets[T.nf] > DEM_MAX_LOOP)
            return fail(h, DEM_E_SHAPE, "shape %d: %d face-loop entries (limit %d)", idx, d.face_offsets[T.nf], DEM_MAX_LOOP);
        double vol6 = 0.0;
        for (int f = 0; f <= T.nf; ++f) T.foff[f] = d.face_offsets[f];
        for (int f = 0; f < T.nf; ++f) {
            const int k0 = T.foff[f], k1 = T.foff[f + 1];
            if (k1 - k0 < 3) return fail(h, DEM_E_SHAPE, "shape %d: face %d has < 3 vertices", idx, f);
            HostVec nrm{0, 0, 0};
            for (int k = k0; k < k1; ++k) {
                int a = d.face_vertices[k];
                if (a < 0 || a >= T.nv) return fail(h, DEM_E_SHAPE, "shape %d: face %d vertex index %d", idx, f, a);
                T.floop[k] = a;
            }
            for (int k = k0; k < k1; ++k) {
                int kn = (k + 1 < k1) ? k + 1 : k0;
                HostVec p{T.v[T.floop[k]][0], T.v[T.floop[k]][1], T.v[T.floop[k]][2]};
                HostVec q{T.v[T.floop[kn]][0], T.v[T.floop[kn]][1], T.v[T.floop[kn]][2]};
                HostVec c = hcross(p, q);
                nrm.x += c.x;
                nrm.y += c.y;
                nrm.z += c.z;
            }
            double nn = std::sqrt(hdot(nrm, nrm));
            if (!(nn > 0.0)) return fail(h, DEM_E_SHAPE, "shape %d: face %d is degenerate", idx, f);
            vol6 += hdot(nrm, HostVec{T.v[T.floop[k0]][0], T.v[T.floop[k0]][1], T.v[T.floop[k0]][2]});
            HostVec n{nrm.x / nn, nrm.y / nn, nrm.z / nn};
            HostVec o{T.v[T.floop[k0]][0], T.v[T.floop[k0]][1], T.v[T.floop[k0]][2]};
            T.fn[f][0] = n.x;
            T.fn[f][1] = n.y;
            T.fn[f][2] = n.z;
            T.fo[f] = hdot(n, o);
            for (int k = k0; k < k1; ++k) {
                HostVec p{T.v[T.floop[k]][0], T.v[T.floop[k]][1], T.v[T.floop[k]][2]};
                if (std::fabs(hdot(n, p) - T.fo[f]) > 1e-9 * (1.0 + R))
                    return fail(h, DEM_E_SHAPE, "shape %d: face %d is not planar", idx, f);
            }
            HostVec e1 = hsub(HostVec{T.v[T.floop[k0 + 1]][0], T.v[T.floop[k0 + 1]][1], T.v[T.floop[k0 + 1]][2]}, o);
            double l1 = std::sqrt(hdot(e1, e1));
            e1 = {e1.x / l1, e1.y / l1, e1.z / l1};
            HostVec e2 = hcross(n, e1);
            T.fe1[f][0] = e1.x;
            T.fe1[f][1] = e1.y;
            T.fe1[f][2] = e1.z;
            bool convex = true;
            for (int k = k0; k < k1; ++k) {
                int kn = (k + 1 < k1) ? k + 1 : k0;
                int kp = (k > k0) ? k - 1 : k1 - 1;
                HostVec a{T.v[T.floop[k]][0], T.v[T.floop[k]][1], T.v[T.floop[k]][2]};
                HostVec b{T.v[T.floop[kn]][0], T.v[T.floop[kn]][1], T.v[T.floop[kn]][2]};
                HostVec c{T.v[T.floop[kp]][0], T.v[T.floop[kp]][1], T.v[T.floop[kp]][2]};
                HostVec ed = hsub(b, a);
                HostVec in = hcross(n, ed);  // inward in-plane normal for a counter-clockwise loop
                T.lnrm[k][0] = in.x;
                T.lnrm[k][1] = in.y;
                T.lnrm[k][2] = in.z;
                T.loff[k] = hdot(in, a);
                T.linv[k] = 1.0 / hdot(ed, ed);
                HostVec ra = hsub(a, o);
                T.lxy[k][0] = hdot(ra, e1);
                T.lxy[k][1] = hdot(ra, e2);
                if (hdot(hcross(hsub(a, c), ed), n) < -1e-12) convex = false;
            }
            T.fconvex[f] = convex ? 1 : 0;
            HostVec c{0, 0, 0};
            for (int k = k0; k < k1; ++k) {
                c.x += T.v[T.floop[k]][0];
                c.y += T.v[T.floop[k]][1];
                c.z += T.v[T.floop[k]][2];
            }
            const double inv = 1.0 / (k1 - k0);
            c = {c.x * inv, c.y * inv, c.z * inv};
            double rad = 0.0;
            for (int k = k0; k < k1; ++k) {
                HostVec dv = hsub(HostVec{T.v[T.floop[k]][0], T.v[T.floop[k]][1], T.v[T.floop[k]][2]}, c);
                rad = std::max(rad, std::sqrt(hdot(dv, dv)));
            }
            T.fc[f][0] = c.x;
            T.fc[f][1] = c.y;
            T.fc[f][2] = c.z;
            T.frad[f] = rad * (1.0 + 1e-6) + 1e-9;  // conservative bounding circle
        }
        if (!(vol6 > 0.0))
            return fail(h, DEM_E_SHAPE, "shape %d: face loops are not counter-clockwise seen from outside", idx);
    }
    support_planes(T, dim);
    return DEM_OK;
}

// ---- shape-local feature cells ----------------------------------------

HostVec hv(const double (&a)[3]) { return {a[0], a[1], a[2]}; }

double seg_dist(HostVec p, HostVec a, HostVec b)
{
    const HostVec d = hsub(b, a), r = hsub(p, a);
    const double dd = hdot(d, d);
    const double s = dd > 0.0 ? std::clamp(hdot(r, d) / dd, 0.0, 1.0) : 0.0;
    const HostVec q = hsub(r, HostVec{s * d.x, s * d.y, s * d.z});
    return std::sqrt(hdot(q, q));
}

// Distance from p to face f, a planar polygon (convex or not): to its plane
// when p projects inside the loop (crossing number in face coordinates),
// else to its nearest loop edge.
double face_dist(const ShapeTab<double> &T, int f, HostVec p)
{
    const int k0 = T.foff[f], k1 = T.foff[f + 1];
    const HostVec n = hv(T.fn[f]), e1 = hv(T.fe1[f]), e2 = hcross(n, e1);
    const double d = hdot(n, p) - T.fo[f];
    const HostVec r = hsub(p, hv(T.v[T.floop[k0]]));
    const double x = hdot(r, e1), y = hdot(r, e2);
    bool in = false;
    for (int k = k0; k < k1; ++k) {
        const int kn = k + 1 < k1 ? k + 1 : k0;
        const double ax = T.lxy[k][0], ay = T.lxy[k][1], bx = T.lxy[kn][0], by = T.lxy[kn][1];
        if ((ay > y) != (by > y) && x < ax + (y - ay) * (bx - ax) / (by - ay)) in = !in;
    }
    if (in) return std::fabs(d);
    double m = 1e300;
    for (int k = k0; k < k1; ++k) {
        const int kn = k + 1 < k1 ? k + 1 : k0;
        m = std::min(m, seg_dist(p, hv(T.v[T.floop[k]]), hv(T.v[T.floop[kn]])));
    }
    return m;
}

// Reach of shape s's cells among the replica's shapes t: a vertex of any
// shape within the cutoff of a feature of s (sigma = r_s + r_max), with room
// for the rounding of FP32 positions; an edge, within that plus the longest
// half edge (the edge is looked up by its midpoint).  L: half width of the
// grid, beyond which no point is within reach of s.
struct FcReach {
    double v, e, L;
};
FcReach fc_reach(const std::vector<ShapeTab<double>> &t, int s)
{
    double rmax = 0.0, Rmax = 0.0, ehmax = 0.0;
    for (const ShapeTab<double> &T : t) {
        rmax = std::max(rmax, T.r);
        Rmax = std::max(Rmax, T.R);
        for (int k = 0; k < T.ne; ++k) ehmax = std::max(ehmax, T.eh[k]);
    }
    const ShapeTab<double> &S = t[s];
    const double rc = kWcaCut * (S.r + rmax);
    const double v = rc * 1.001 + 1e-4 * (S.R + Rmax + rc);
    return {v, v + ehmax, S.R + v + ehmax};
}

// Grid geometry of every shape's cells, in both precisions' tables.
void fc_geometry(std::vector<ShapeTab<double>> &t64, std::vector<ShapeTab<float>> &t32, int dim)
{
    for (size_t s = 0; s < t64.size(); ++s) {
        const FcReach q = fc_reach(t64, (int)s);
        const int g = dim == 3 ? kFcGrid3 : kFcGrid2;
        t64[s].fc_g = t32[s].fc_g = g;
        t64[s].fc_lo = -q.L;
        t64[s].fc_ih = g / (2.0 * q.L);
        t32[s].fc_lo = (float)t64[s].fc_lo;
        t32[s].fc_ih = (float)t64[s].fc_ih;
    }
}

// The cells of shape s (kFcCells entries; see kFcGrid3): each cell keeps
// the features whose distance from its centre is within reach plus its half
// diagonal, so every point of the cell is covered.
void fc_build(const std::vector<ShapeTab<double>> &t, int s, int dim, uint2 *cells)
{
    const ShapeTab<double> &T = t[s];
    const FcReach q = fc_reach(t, s);
    const int g = T.fc_g;
    const double w = 1.0 / T.fc_ih, hd = 0.5 * w * std::sqrt((double)dim);
    for (int c = 0; c < kFcCells; ++c) cells[c] = make_uint2(0u, 0u);
    for (int iz = 0; iz < (dim == 3 ? g : 1); ++iz)
        for (int iy = 0; iy < g; ++iy)
            for (int ix = 0; ix < g; ++ix) {
                const HostVec c{T.fc_lo + (ix + 0.5) * w, T.fc_lo + (iy + 0.5) * w,
                                dim == 3 ? T.fc_lo + (iz + 0.5) * w : 0.0};
                unsigned fm = 0u, em = 0u;
                if (dim == 3) {
                    for (int f = 0; f < T.nf; ++f)
                        if (face_dist(T, f, c) <= q.v + hd) fm |= 1u << f;
                    for (int k = 0; k < T.ne; ++k)
                        if (seg_dist(c, hv(T.v[T.e[k][0]]), hv(T.v[T.e[k][1]])) <= q.e + hd) em |= 1u << k;
                } else {
                    for (int k = 0; k < T.ne; ++k)
                        if (seg_dist(c, hv(T.v[T.e[k][0]]), hv(T.v[T.e[k][1]])) <= q.v + hd) fm |= 1u << k;
                }
                cells[(iz * g + iy) * g + ix] = make_uint2(fm, em);
            }
}

void to_float(const ShapeTab<double> &D, ShapeTab<float> &F)
{
    std::memset(&F, 0, sizeof F);
    F.nv = D.nv;
    F.ne = D.ne;
    F.nf = D.nf;
    F.r = (float)D.r;
    F.R = (float)D.R;
    for (int k = 0; k < DEM_MAX_VERTS; ++k)
        for (int a = 0; a < 3; ++a) F.v[k][a] = (float)D.v[k][a];
    for (int k = 0; k < DEM_MAX_EDGES; ++k) {
        F.e[k][0] = D.e[k][0];
        F.e[k][1] = D.e[k][1];
        for (int a = 0; a < 3; ++a) {
            F.ed[k][a] = (float)D.ed[k][a];
            F.em[k][a] = (float)D.em[k][a];
        }
        F.eh[k] = (float)(D.eh[k] * (1.0 + 1e-6));  // keep the FP32 bounds conservative
        F.el2[k] = (float)D.el2[k];
        F.einv[k] = (float)D.einv[k];
    }
    for (int f = 0; f <= DEM_MAX_FACES; ++f) F.foff[f] = D.foff[f];
    for (int f = 0; f < DEM_MAX_FACES; ++f) {
        F.fconvex[f] = D.fconvex[f];
        F.fo[f] = (float)D.fo[f];
        F.frad[f] = (float)(D.frad[f] * (1.0 + 1e-6));
        for (int a = 0; a < 3; ++a) {
            F.fn[f][a] = (float)D.fn[f][a];
            F.fe1[f][a] = (float)D.fe1[f][a];
            F.fc[f][a] = (float)D.fc[f][a];
        }
    }
    for (int k = 0; k < DEM_MAX_LOOP; ++k) {
        F.floop[k] = D.floop[k];
        for (int a = 0; a < 3; ++a) F.lnrm[k][a] = (float)D.lnrm[k][a];
        F.loff[k] = (float)D.loff[k];
        F.linv[k] = (float)D.linv[k];
        F.lxy[k][0] = (float)D.lxy[k][0];
        F.lxy[k][1] = (float)D.lxy[k][1];
    }
    F.nsep = D.nsep;
    for (int k = 0; k < kMaxSep; ++k) {
        for (int a = 0; a < 3; ++a) F.sn[k][a] = (float)D.sn[k][a];
        float o = (float)D.so[k];  // rounded up, so the FP32 plane still bounds the body
        if ((double)o < D.so[k]) o = std::nextafter(o, 3.0e38f);
        F.so[k] = o;
    }
}

int auto_capacity(const dem_params &p, double rl)
{
    double vol = p.dim == 3 ? p.box[0] * p.box[1] * p.box[2] : p.box[0] * p.box[1];
    double dens = vol > 0.0 ? (double)p.n / vol : 0.0;
    double expect = p.dim == 3 ? dens * 4.0 / 3.0 * M_PI * rl * rl * rl : dens * M_PI * rl * rl;
    int cap = (int)std::ceil(1.8 * expect) + 16;
    cap = std::max(16, std::min(cap, (int)std::max<int64_t>(p.n, 16)));
    return std::min(kRowMax, (cap + 3) & ~3);
}


size_t rec_bytes(int precision) { return precision == DEM_FP32 ? sizeof(SlotRec<float>) : sizeof(SlotRec<double>); }
size_t partrec_bytes(int precision) { return precision == DEM_FP32 ? sizeof(PartRec<float>) : sizeof(PartRec<double>); }

void drop_graph(dem_system *h)
{
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->gexec_multi) (void)hipGraphExecDestroy(h->gexec_multi);
    if (h->graph_multi) (void)hipGraphDestroy(h->graph_multi);
    h->gexec = h->gexec_multi = nullptr;
    h->graph = h->graph_multi = nullptr;
}

Launch make_launch(const dem_system *h)
{
    Launch L;
    L.b = h->bp;
    L.reps = h->d_reps;
    L.s = h->st;
    L.o = h->out;
    L.l = h->lst;
    L.l.chunk_rep = h->d_chunk_rep;
    L.f.rot = h->rot;
    L.f.rec64 = h->rec64;
    L.f.rec = h->rec;
    L.f.tab = h->precision == DEM_FP32 ? h->tab32 : h->tab64;
    L.f.tab64 = h->tab64;
    L.precision = h->precision;
    L.ke_part = h->ke_part;
    L.thermo = h->thermo;
    L.budget = h->budget;
    L.steps = h->steps;
    return L;
}

int tiles_of(int pcap, int tile) { return (pcap + tile - 1) / tile; }

// Batch-wide launch parameters from the replica table.
void refresh_batch(dem_system *h)
{
    BatchParams &b = h->bp;
    b.nrep = 0;
    b.tab_slots = 1;
    b.pair_lanes = h->pair_lanes;
    b.pair_waves = h->pair_waves;
    b.pair_sep = h->pair_sep;
    b.pair_split = h->pair_split;
    b.feature_cells = h->feature_cells;
    b.tile = pair_tile(h->pair_sep);
    long long tiles = 0;
    for (size_t r = 0; r < h->reps.size(); ++r) {
        const Replica &R = h->reps[r];
        if (!R.live) continue;
        b.nrep = (int)r + 1;
        b.tab_slots = std::max(b.tab_slots, R.sp.n_shapes);
        tiles += tiles_of(R.sp.pcap, b.tile);
    }
    b.nchunk = h->chunks.high();
    b.dim = h->dim;
    // by default one round of blocks, as many as the device holds at once
    // (a second round adds a whole block's latency but evens out the
    // tail), no more than the tiles use
    const int stage = b.pair_split ? kForces : kFused;
    const long long resident = (long long)pair_blocks_resident(h->precision, h->dim, b.tab_slots, b.pair_lanes,
                                                               b.pair_waves, b.pair_sep, stage, b.feature_cells) *
                               h->pair_grid;
    // the split form's force kernel takes units of kPairWaves * 64 / lanes
    // compacted pairs, at most one per that many pair slots
    const long long units = tiles * b.tile / (kPairWaves * (64 / b.pair_lanes)) + b.nrep;
    const long long want = std::max<long long>(8, std::min<long long>(b.pair_split ? units : tiles, resident));
    b.pair_blocks = (int)((want + 7) / 8 * 8);
    b.search_blocks = 8;
    if (b.pair_split) {
        const long long rs = pair_blocks_resident(h->precision, h->dim, b.tab_slots, b.pair_lanes, b.pair_waves,
                                                  b.pair_sep, kSearchOnly, 0);
        b.search_blocks = (int)((std::max<long long>(8, std::min(tiles, rs)) + 7) / 8 * 8);
    }
}

// Pair slots of every replica follow its particle slots: cap / 2 per slot.
void place_pairs(dem_system *h)
{
    for (Replica &R : h->reps) {
        R.sp.poff = (int)((int64_t)R.chunk0 * kChunk * h->bp.cap / 2);
        R.sp.pcap = (int)((int64_t)R.nchunks * kChunk * h->bp.cap / 2);
    }
}

// The box and cell geometry of the NPT replicas, which the device moves on
// every step, read back into the host copies (synchronises).
dem_status sync_dynamic(dem_system *h)
{
    bool any = false;
    for (const Replica &R : h->reps) any |= R.live && R.on_device && R.sp.ensemble == DEM_NPT;
    if (!any) return DEM_OK;
    std::vector<SysParams> dev(h->reps.size());
    HIPCHK(h, hipMemcpyAsync(dev.data(), h->d_reps, sizeof(SysParams) * dev.size(), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (size_t r = 0; r < h->reps.size(); ++r) {
        SysParams &sp = h->reps[r].sp;
        if (!h->reps[r].live || !h->reps[r].on_device || sp.ensemble != DEM_NPT) continue;
        const SysParams &d = dev[r];
        for (int a = 0; a < 3; ++a) {
            sp.box[a] = d.box[a];
            sp.cellw[a] = d.cellw[a];
            sp.nc[a] = d.nc[a];
            sp.box_build[a] = d.box_build[a];
        }
        sp.ncell = d.ncell;
        sp.use_cells = d.use_cells;
    }
    return DEM_OK;
}

dem_status upload_tables(dem_system *h)
{
    if (dem_status st = sync_dynamic(h); st != DEM_OK) return st;
    std::vector<SysParams> sp(h->reps.size());
    for (size_t r = 0; r < h->reps.size(); ++r) {
        sp[r] = h->reps[r].sp;
        sp[r].live = h->reps[r].live ? 1 : 0;
        sp[r].rid = (int)r;
    }
    h->h_chunk_rep.assign((size_t)h->chunks.size(), -1);
    for (size_t r = 0; r < h->reps.size(); ++r) {
        const Replica &R = h->reps[r];
        if (!R.live) continue;
        for (int c = R.chunk0; c < R.chunk0 + R.nchunks; ++c) h->h_chunk_rep[c] = (int32_t)r;
    }
    // in stream order, so kernels already queued see the old tables; the
    // host sources must live until the copies are done
    HIPCHK(h, hipMemcpyAsync(h->d_reps, sp.data(), sizeof(SysParams) * sp.size(), hipMemcpyHostToDevice, h->stream));
    if (!h->h_chunk_rep.empty())
        HIPCHK(h, hipMemcpyAsync(h->d_chunk_rep, h->h_chunk_rep.data(), sizeof(int32_t) * h->h_chunk_rep.size(),
                                 hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (Replica &R : h->reps) R.on_device = R.live;
    refresh_batch(h);
    drop_graph(h);
    return DEM_OK;
}

// Row storage and everything sized by the row capacity: rows, pair entries
// and pair records.  Rows keep their contents (row k of particle i sits at
// k * N + i whatever the capacity); the pair entries, whose slots move with
// the capacity, are written again from the rows, so the lists do not change.
dem_status alloc_nbr(dem_system *h, int cap)
{
    if (cap > kRowMax) return fail(h, DEM_E_CAPACITY, "neighbour rows of %d exceed the limit %d", cap, kRowMax);
    (void)hipStreamSynchronize(h->stream);
    const size_t N = (size_t)std::max(h->Ncap, kChunk);
    const size_t maxp = N * (size_t)cap / 2;
    if (maxp > (size_t)INT32_MAX) return fail(h, DEM_E_ARG, "pair capacity overflows int32");
    int32_t *nbr = nullptr;
    if (hipMalloc(&nbr, sizeof(int32_t) * (size_t)cap * N) != hipSuccess)
        return fail(h, DEM_E_OOM, "neighbour list of %d x %zu entries", cap, N);
    if (h->lst.nbr && h->bp.cap > 0)
        HIPCHK(h, hipMemcpyAsync(nbr, h->lst.nbr, sizeof(int32_t) * (size_t)std::min(cap, h->bp.cap) * N,
                                 hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    (void)hipFree(h->lst.nbr);
    (void)hipFree(h->lst.pairs);
    (void)hipFree(h->lst.cpairs);
    (void)hipFree(h->rec);
    (void)hipFree(h->lst.smask);
    h->lst.nbr = nbr;
    h->lst.pairs = nullptr;
    h->lst.cpairs = nullptr;
    h->rec = nullptr;
    h->lst.smask = nullptr;
    if (hipMalloc(&h->lst.pairs, sizeof(int4) * maxp) != hipSuccess ||
        hipMalloc(&h->lst.cpairs, sizeof(int4) * maxp) != hipSuccess ||
        hipMalloc(&h->rec, rec_bytes(h->precision) * (size_t)cap * N) != hipSuccess ||
        hipMalloc(&h->lst.smask, sizeof(uint32_t) * (size_t)slot_words(cap) * N) != hipSuccess)
        return fail(h, DEM_E_OOM, "neighbour list of %d x %zu entries", cap, N);
    // records never written read as zeros (stamp 0, no force); no slot written yet
    HIPCHK(h, hipMemsetAsync(h->rec, 0, rec_bytes(h->precision) * (size_t)cap * N, h->stream));
    HIPCHK(h, hipMemsetAsync(h->lst.smask, 0, sizeof(uint32_t) * (size_t)slot_words(cap) * N, h->stream));
    h->bp.cap = cap;
    place_pairs(h);
    dem_status st = upload_tables(h);
    if (st != DEM_OK) return st;
    launch_lists(make_launch(h), LISTS_REFILL, h->stream);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return DEM_OK;
}

dem_status alloc_core(dem_system *h, int Ncap, int Ccap, int Scap, int Rcap)
{
    h->Ncap = Ncap;
    const size_t N = (size_t)std::max(Ncap, kChunk);
    const size_t nch = N / kChunk;
    h->chunks.reset(Ncap / kChunk);
    h->cells.reset(Ccap);
    h->shapes.reset(Scap);
    h->reps.assign((size_t)Rcap, Replica{});
    h->bp.N = (int)N;
    bool ok = hipMalloc(&h->d_reps, sizeof(SysParams) * Rcap) == hipSuccess &&
              hipMalloc(&h->d_chunk_rep, sizeof(int32_t) * nch) == hipSuccess &&
              hipMalloc(&h->tab64, sizeof(ShapeTab<double>) * Scap) == hipSuccess &&
              hipMalloc(&h->tab32, sizeof(ShapeTab<float>) * Scap) == hipSuccess &&
              hipMalloc(&h->fcells, sizeof(uint2) * kFcCells * Scap) == hipSuccess &&
              hipMalloc(&h->ke_part, sizeof(double) * kKePer * nch) == hipSuccess &&
              hipMalloc(&h->e_part, sizeof(double) * 12 * nch) == hipSuccess &&
              hipMalloc(&h->thermo, sizeof(double) * TH_COUNT * Rcap) == hipSuccess &&
              hipMalloc(&h->budget, sizeof(int64_t) * Rcap) == hipSuccess &&
              hipMalloc(&h->steps, sizeof(int64_t) * Rcap) == hipSuccess &&
              hipMalloc(&h->stats, sizeof(unsigned long long) * ST_COUNT) == hipSuccess &&
              hipMalloc(&h->lst.flags, sizeof(int32_t) * FLAG_COUNT * Rcap) == hipSuccess &&
              hipMalloc(&h->lst.gflags, sizeof(int32_t) * G_COUNT) == hipSuccess &&
              hipMalloc(&h->lst.tile_start, sizeof(int32_t) * (Rcap + 1)) == hipSuccess &&
              hipMalloc(&h->lst.ccount, sizeof(int32_t) * split_words(Rcap)) == hipSuccess &&
              hipMalloc(&h->lst.cell_count, sizeof(int32_t) * std::max(Ccap, 1)) == hipSuccess &&
              hipMalloc(&h->lst.cell_slot, sizeof(int32_t) * kCellCap * (size_t)std::max(Ccap, 1)) == hipSuccess &&
              hipMalloc(&h->lst.pcell, sizeof(int32_t) * N) == hipSuccess &&
              hipMalloc(&h->lst.n_nbr, sizeof(int32_t) * N) == hipSuccess &&
              hipMalloc(&h->lst.xlast, sizeof(double) * 3 * N) == hipSuccess &&
              hipMalloc(&h->lst.klo, sizeof(int32_t) * N) == hipSuccess &&
              hipMalloc(&h->lst.pstart, sizeof(int32_t) * N) == hipSuccess &&
              hipMalloc(&h->lst.ptot, sizeof(int32_t) * (N / lb_rows_per_group + 1)) == hipSuccess &&
              hipMalloc(&h->rot, partrec_bytes(h->precision) * N) == hipSuccess &&
              (h->precision != DEM_FP32 || hipMalloc(&h->rec64, sizeof(PartRec64) * N) == hipSuccess);
    if (!ok) return fail(h, DEM_E_OOM, "device allocation failed");
    h->lst.fcells = h->fcells;
    h->lst.cunit = h->lst.ccount + Rcap;
    h->lst.ctick = h->lst.cunit + Rcap + 1;
    if (h->batch) {  // the batch's own state and output arrays
        double **d[] = {&h->st.x,  &h->st.y,  &h->st.z,  &h->st.qw, &h->st.qx, &h->st.qy, &h->st.qz,
                        &h->st.vx, &h->st.vy, &h->st.vz, &h->st.Lx, &h->st.Ly, &h->st.Lz, &h->out.Fx,
                        &h->out.Fy, &h->out.Fz, &h->out.Tx, &h->out.Ty, &h->out.Tz, &h->out.U};
        for (double **p : d)
            if (hipMalloc(p, sizeof(double) * N) != hipSuccess) return fail(h, DEM_E_OOM, "device allocation failed");
        if (hipMalloc(&h->out.W, sizeof(double) * 9 * N) != hipSuccess ||
            hipMalloc(&h->st.sid, sizeof(int32_t) * N) != hipSuccess ||
            hipMalloc(&h->st.image, sizeof(int32_t) * 3 * N) != hipSuccess)
            return fail(h, DEM_E_OOM, "device allocation failed");
        HIPCHK(h, hipMemsetAsync(h->st.sid, 0, sizeof(int32_t) * N, h->stream));
        h->bp.wstride = (int)N;
        h->bp.nstate = (int)N;
    }
    // initial contents (not captured: plain memsets are fine here)
    HIPCHK(h, hipMemsetAsync(h->lst.flags, 0, sizeof(int32_t) * FLAG_COUNT * Rcap, h->stream));
    HIPCHK(h, hipMemsetAsync(h->lst.gflags, 0, sizeof(int32_t) * G_COUNT, h->stream));
    HIPCHK(h, hipMemsetAsync(h->lst.tile_start, 0, sizeof(int32_t) * (Rcap + 1), h->stream));
    // compacted-pair counts and tickets start at zero; the split form's
    // last workgroups return them to zero after each evaluation
    HIPCHK(h, hipMemsetAsync(h->lst.ccount, 0, sizeof(int32_t) * split_words(Rcap), h->stream));
    HIPCHK(h, hipMemsetAsync(h->lst.cell_count, 0, sizeof(int32_t) * std::max(Ccap, 1), h->stream));
    // rows, pair offsets and cells start empty, so a pass over a replica that
    // has no lists yet reads zeros
    HIPCHK(h, hipMemsetAsync(h->lst.n_nbr, 0, sizeof(int32_t) * N, h->stream));
    HIPCHK(h, hipMemsetAsync(h->lst.klo, 0, sizeof(int32_t) * N, h->stream));
    HIPCHK(h, hipMemsetAsync(h->lst.pstart, 0, sizeof(int32_t) * N, h->stream));
    HIPCHK(h, hipMemsetAsync(h->lst.ptot, 0, sizeof(int32_t) * (N / lb_rows_per_group + 1), h->stream));
    HIPCHK(h, hipMemsetAsync(h->lst.pcell, 0, sizeof(int32_t) * N, h->stream));
    HIPCHK(h, hipMemsetAsync(h->stats, 0, sizeof(unsigned long long) * ST_COUNT, h->stream));
    HIPCHK(h, hipMemsetAsync(h->ke_part, 0, sizeof(double) * kKePer * nch, h->stream));
    HIPCHK(h, hipMemsetAsync(h->budget, 0, sizeof(int64_t) * Rcap, h->stream));
    HIPCHK(h, hipMemsetAsync(h->steps, 0, sizeof(int64_t) * Rcap, h->stream));
    return DEM_OK;
}

void free_all(dem_system *h)
{
    drop_graph(h);
    void *ptrs[] = {h->d_reps, h->d_chunk_rep, h->tab64, h->tab32, h->fcells, h->ke_part, h->e_part, h->thermo, h->budget,
                    h->steps, h->stats, h->lst.flags, h->lst.gflags, h->lst.tile_start, h->lst.ccount, h->lst.cell_count,
                    h->lst.cell_slot, h->lst.pcell, h->lst.n_nbr, h->lst.xlast, h->lst.klo,
                    h->lst.pstart, h->lst.ptot, h->lst.nbr, h->lst.pairs, h->lst.cpairs, h->lst.smask, h->rot, h->rec,
                    h->rec64};
    for (void *p : ptrs) (void)hipFree(p);
    if (h->batch) {
        void *own[] = {h->st.x,  h->st.y,  h->st.z,  h->st.qw, h->st.qx,  h->st.qy,  h->st.qz,  h->st.vx,
                       h->st.vy, h->st.vz, h->st.Lx, h->st.Ly, h->st.Lz,  h->st.sid, h->st.image, h->out.Fx,
                       h->out.Fy, h->out.Fz, h->out.Tx, h->out.Ty, h->out.Tz, h->out.U, h->out.W};
        for (void *p : own) (void)hipFree(p);
    }
}

dem_status latched(dem_system *h)
{
    std::vector<int32_t> flags((size_t)FLAG_COUNT * h->reps.size());
    HIPCHK(h, hipMemcpyAsync(flags.data(), h->lst.flags, sizeof(int32_t) * flags.size(), hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (size_t r = 0; r < h->reps.size(); ++r) {
        if (!h->reps[r].live) continue;
        const int32_t *f = flags.data() + FLAG_COUNT * r;
        if (f[FLAG_NONFINITE]) return fail(h, DEM_E_NONFINITE, "replica %zu: non-finite position or velocity", r);
        if (f[FLAG_CELLOVF])
            return fail(h, DEM_E_CAPACITY, "replica %zu: a cell held more than %d particles in a list build", r,
                        kCellCap);
        if (f[FLAG_MAXROW] > h->bp.cap)
            return fail(h, DEM_E_CAPACITY, "replica %zu: neighbour row of %d exceeds capacity %d", r, f[FLAG_MAXROW],
                        h->bp.cap);
        if (f[FLAG_BOXSMALL])
            return fail(h, DEM_E_STATE, "replica %zu: the barostat shrank the box below twice the list radius", r);
    }
    return DEM_OK;
}

void enqueue_step(dem_system *h, hipStream_t s)
{
    const Launch L = make_launch(h);
    launch_kick_drift(L, s);
    launch_pairs(L, h->counting ? h->stats : nullptr, s);
    launch_gather(L, true, s);
}

// Steps per launch of the long graph: consecutive graph launches leave a
// gap of several microseconds on the device, which a chain of steps in one
// graph does not.
constexpr int kGraphSteps = 8;

dem_status capture_steps(dem_system *h, int steps, hipGraph_t *graph, hipGraphExec_t *exec)
{
    HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < steps; ++k) enqueue_step(h, h->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    if (e != hipSuccess || !g) return fail(h, DEM_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    *graph = g;
    HIPCHK(h, hipGraphInstantiate(exec, g, nullptr, nullptr, 0));
    return DEM_OK;
}

dem_status ensure_graph(dem_system *h)
{
    if (h->gexec && h->gexec_multi) return DEM_OK;
    drop_graph(h);
    dem_status st = capture_steps(h, 1, &h->graph, &h->gexec);
    if (st == DEM_OK) st = capture_steps(h, kGraphSteps, &h->graph_multi, &h->gexec_multi);
    return st;
}

// Builds the lists of replica `only` (all live replicas if LISTS_ALL) from
// the current positions, now, growing the row capacity while rows overflow
// and the capacity is automatic.  Other replicas' lists, and any rebuild
// their next step has pending, are left as they are.
dem_status build_lists_sync(dem_system *h, int only)
{
    for (int attempt = 0; attempt < 4; ++attempt) {
        for (size_t r = 0; r < h->reps.size(); ++r) {
            if (!h->reps[r].live || (only >= 0 && (int)r != only)) continue;
            k_set_i32<<<1, 1, 0, h->stream>>>(h->lst.flags + FLAG_COUNT * r + FLAG_MAXROW, 0);
        }
        launch_lists(make_launch(h), only, h->stream);
        HIPCHK(h, hipGetLastError());
        std::vector<int32_t> flags((size_t)FLAG_COUNT * h->reps.size());
        HIPCHK(h, hipMemcpyAsync(flags.data(), h->lst.flags, sizeof(int32_t) * flags.size(), hipMemcpyDeviceToHost,
                                 h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        int maxrow = 0;
        for (size_t r = 0; r < h->reps.size(); ++r) {
            if (!h->reps[r].live || (only >= 0 && (int)r != only)) continue;
            if (flags[FLAG_COUNT * r + FLAG_CELLOVF])
                return fail(h, DEM_E_CAPACITY, "replica %zu: a cell holds more than %d particles", r, kCellCap);
            maxrow = std::max(maxrow, flags[FLAG_COUNT * r + FLAG_MAXROW]);
        }
        if (maxrow <= h->bp.cap) {
            for (size_t r = 0; r < h->reps.size(); ++r)
                if (h->reps[r].live && (only < 0 || (int)r == only)) {
                    k_count_build<<<1, 1, 0, h->stream>>>(h->lst.flags + FLAG_COUNT * r);
                    k_box_built<<<1, 1, 0, h->stream>>>(h->d_reps, (int)r);
                }
            HIPCHK(h, hipGetLastError());
            return DEM_OK;
        }
        if (!h->auto_cap)
            return fail(h, DEM_E_CAPACITY, "neighbour row of %d exceeds capacity %d", maxrow, h->bp.cap);
        dem_status st = alloc_nbr(h, std::min(kRowMax, ((maxrow * 5) / 4 + 8 + 3) & ~3));
        if (st != DEM_OK) return st;
    }
    return fail(h, DEM_E_CAPACITY, "neighbour capacity did not converge");
}

// Validates params against the handle and builds the replica's tables and
// parameters (everything but its slots).
dem_status describe_replica(dem_system *h, const dem_params &p, Replica &R, std::vector<ShapeTab<double>> &t64,
                            std::vector<ShapeTab<float>> &t32)
{
    if (p.dim != 2 && p.dim != 3) return fail(h, DEM_E_ARG, "dim must be 2 or 3");
    if (p.dim != h->dim) return fail(h, DEM_E_ARG, "replica dim %d differs from the batch's %d", p.dim, h->dim);
    if (p.precision != h->precision) return fail(h, DEM_E_ARG, "replica precision differs from the batch's");
    if (p.n < 0 || p.n > (int64_t)INT32_MAX / 64) return fail(h, DEM_E_ARG, "n out of range");
    if (p.n_shapes < 1 || p.n_shapes > DEM_MAX_SHAPES || !p.shapes)
        return fail(h, DEM_E_ARG, "n_shapes must be 1..%d", DEM_MAX_SHAPES);
    if (p.ensemble != DEM_NVE && p.ensemble != DEM_NVT && p.ensemble != DEM_NPT) return fail(h, DEM_E_ARG, "bad ensemble");
    if (p.list_mode != DEM_LISTS_AUTO && p.list_mode != DEM_LISTS_MULTI) return fail(h, DEM_E_ARG, "bad list_mode");
    if (!(p.dt > 0.0) || !(p.skin >= 0.0) || !(p.rebuild_frac > 0.0) || !(p.epsilon > 0.0) || !(p.parallel_sin2 >= 0.0))
        return fail(h, DEM_E_ARG, "dt, epsilon, rebuild_frac must be > 0; skin, parallel_sin2 >= 0");
    if (p.ensemble == DEM_NVT && (!(p.kT > 0.0) || !(p.tau_T > 0.0)))
        return fail(h, DEM_E_ARG, "NVT needs kT > 0 and tau_T > 0");
    if (p.ensemble == DEM_NPT && (!(p.kT > 0.0) || !(p.tau_T > 0.0) || !(p.tau_P > 0.0) || !(p.pressure >= 0.0) ||
                                  p.n < 2))
        return fail(h, DEM_E_ARG, "NPT needs kT, tau_T, tau_P > 0, pressure >= 0 and at least 2 particles");
    for (int a = 0; a < p.dim; ++a)
        if (!(p.box[a] > 0.0)) return fail(h, DEM_E_ARG, "box must be positive");
    R = Replica{};
    R.prm = p;
    R.prm.shapes = nullptr;
    t64.assign((size_t)p.n_shapes, ShapeTab<double>{});
    t32.assign((size_t)p.n_shapes, ShapeTab<float>{});
    double Rmax = 0.0, rmax = 0.0;
    SysParams &sp = R.sp;
    std::memset(&sp, 0, sizeof sp);
    for (int s = 0; s < p.n_shapes; ++s) {
        dem_status st = build_table(h, s, p.shapes[s], p.dim, t64[s]);
        if (st != DEM_OK) return st;
        to_float(t64[s], t32[s]);
        sp.mass[s] = p.shapes[s].mass;
        for (int a = 0; a < 3; ++a) sp.inertia[s][a] = (p.dim == 2 && a < 2) ? 0.0 : p.shapes[s].inertia[a];
        sp.R[s] = t64[s].R;
        sp.rad[s] = p.shapes[s].rounding_radius;
        Rmax = std::max(Rmax, t64[s].R);
        rmax = std::max(rmax, p.shapes[s].rounding_radius);
    }
    fc_geometry(t64, t32, p.dim);
    // r_list = 2 R_max + 2^(1/6) sigma_max + skin
    const double rl = 2.0 * Rmax + kWcaCut * (2.0 * rmax) + p.skin;
    R.r_list = rl;
    sp.n = (int)p.n;
    sp.dim = p.dim;
    sp.n_shapes = p.n_shapes;
    sp.ensemble = p.ensemble;
    sp.use_cells = 1;
    for (int a = 0; a < 3; ++a) {
        sp.box[a] = (a < p.dim) ? p.box[a] : 1.0;
        if (a < p.dim) {
            if (p.box[a] < 2.0 * rl)
                return fail(h, DEM_E_ARG, "box %g on axis %d is below 2 r_list = %g", p.box[a], a, 2.0 * rl);
            sp.nc[a] = (int)std::floor(p.box[a] / rl);
            if (sp.nc[a] < 3) sp.use_cells = 0;
        } else {
            sp.nc[a] = 1;
        }
        sp.cellw[a] = sp.box[a] / (double)sp.nc[a];
    }
    sp.ncell = sp.nc[0] * sp.nc[1] * sp.nc[2];
    sp.rl2 = rl * rl;
    sp.disp2 = (p.rebuild_frac * p.skin) * (p.rebuild_frac * p.skin);
    sp.eps = p.epsilon;
    sp.par_s2 = p.parallel_sin2;
    sp.dt = p.dt;
    sp.kT = p.kT;
    const int drot = p.dim == 2 ? 1 : 3;
    sp.g = (double)(p.dim * p.n + drot * p.n - p.dim);
    sp.rlist = rl;
    for (int a = 0; a < 3; ++a) {
        sp.nc0[a] = sp.nc[a];
        sp.box_build[a] = sp.box[a];
    }
    if (p.ensemble == DEM_NPT) {
        // Sec. IV.C barostat: N_f = d (n - 1) translational degrees of
        // freedom, alpha = 1 + d / N_f, W = (N_f + d) kT tau_P^2; the
        // thermostat also takes the barostat's degree of freedom
        const double Nf = (double)(p.dim * (p.n - 1));
        sp.alpha = 1.0 + p.dim / Nf;
        sp.Wm = (Nf + p.dim) * p.kT * p.tau_P * p.tau_P;
        sp.pext = p.pressure;
        sp.g += 1.0;
    }
    sp.Qm = sp.g * p.kT * p.tau_T * p.tau_T;
    return DEM_OK;
}

// Takes slots for a described replica, uploads its tables, copies its state
// in (a batch) and checks its shape ids.  Returns the slot in *rid.
dem_status place_replica(dem_system *h, Replica &R, const std::vector<ShapeTab<double>> &t64,
                         const std::vector<ShapeTab<float>> &t32, const dem_state_ptrs *src, int *rid)
{
    int slot = -1;
    for (size_t r = 0; r < h->reps.size(); ++r)
        if (!h->reps[r].live) {
            slot = (int)r;
            break;
        }
    if (slot < 0) return fail(h, DEM_E_OOM, "no free replica slot (%zu in use)", h->reps.size());
    const int n = R.sp.n;
    R.nchunks = (n + kChunk - 1) / kChunk;
    R.ncells = R.sp.ncell;
    R.nshapes = R.sp.n_shapes;
    R.chunk0 = h->chunks.find(R.nchunks);
    R.cell0 = h->cells.find(R.ncells);
    R.shape0 = h->shapes.find(R.nshapes);
    if (R.chunk0 < 0) return fail(h, DEM_E_OOM, "no run of %d free particle slots", R.nchunks * kChunk);
    if (R.cell0 < 0) return fail(h, DEM_E_OOM, "no run of %d free cell slots", R.ncells);
    if (R.shape0 < 0) return fail(h, DEM_E_OOM, "no run of %d free shape slots", R.nshapes);
    R.sp.off = R.chunk0 * kChunk;
    R.sp.coff = R.cell0;
    R.sp.sbase = R.shape0;
    R.sp.rid = slot;
    const size_t off = (size_t)R.sp.off;
    if (n > 0 && h->batch) {  // copy the replica's state into the batch's arrays
        const double *from[] = {src->x,  src->y,  src->qw, src->qx, src->qy, src->qz,
                                src->vx, src->vy, src->vz, src->Lx, src->Ly, src->Lz};
        double *to[] = {h->st.x, h->st.y, h->st.qw, h->st.qx, h->st.qy, h->st.qz,
                        h->st.vx, h->st.vy, h->st.vz, h->st.Lx, h->st.Ly, h->st.Lz};
        for (int k = 0; k < 12; ++k) {
            if (!from[k]) return fail(h, DEM_E_ARG, "null state array");
            HIPCHK(h, hipMemcpyAsync(to[k] + off, from[k], sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
        }
        if (h->dim == 3) {
            if (!src->z) return fail(h, DEM_E_ARG, "null state array");
            HIPCHK(h, hipMemcpyAsync(h->st.z + off, src->z, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
        } else {
            HIPCHK(h, hipMemsetAsync(h->st.z + off, 0, sizeof(double) * n, h->stream));
        }
        if (!src->shape_id || !src->image) return fail(h, DEM_E_ARG, "null state array");
        HIPCHK(h, hipMemcpyAsync(h->st.sid + off, src->shape_id, sizeof(int32_t) * n, hipMemcpyDeviceToDevice,
                                 h->stream));
        HIPCHK(h, hipMemcpyAsync(h->st.image + 3 * off, src->image, sizeof(int32_t) * 3 * n,
                                 hipMemcpyDeviceToDevice, h->stream));
    }
    if (n > 0) {  // shape ids index the LDS tables: validate before any kernel reads them
        std::vector<int32_t> sid((size_t)n);
        HIPCHK(h, hipMemcpyAsync(sid.data(), h->st.sid + off, sizeof(int32_t) * n, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        for (int i = 0; i < n; ++i)
            if (sid[i] < 0 || sid[i] >= R.sp.n_shapes)
                return fail(h, DEM_E_ARG, "shape_id[%d] = %d outside [0, %d)", i, sid[i], R.sp.n_shapes);
    }
    HIPCHK(h, hipMemcpyAsync(static_cast<ShapeTab<double> *>(h->tab64) + R.shape0, t64.data(),
                             sizeof(ShapeTab<double>) * R.nshapes, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(static_cast<ShapeTab<float> *>(h->tab32) + R.shape0, t32.data(),
                             sizeof(ShapeTab<float>) * R.nshapes, hipMemcpyHostToDevice, h->stream));
    {
        std::vector<uint2> cells((size_t)kFcCells * R.nshapes);
        for (int s = 0; s < R.nshapes; ++s) fc_build(t64, s, R.sp.dim, cells.data() + (size_t)s * kFcCells);
        HIPCHK(h, hipMemcpyAsync(h->fcells + (size_t)R.shape0 * kFcCells, cells.data(), sizeof(uint2) * cells.size(),
                                 hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));  // the host cells go out of scope
    }
    HIPCHK(h, hipMemsetAsync(h->lst.cell_count + R.cell0, 0, sizeof(int32_t) * R.ncells, h->stream));
    HIPCHK(h, hipMemsetAsync(h->lst.flags + FLAG_COUNT * slot, 0, sizeof(int32_t) * FLAG_COUNT, h->stream));
    if (n > 0) {  // the slots' previous owner left its lists there
        HIPCHK(h, hipMemsetAsync(h->lst.n_nbr + off, 0, sizeof(int32_t) * n, h->stream));
        HIPCHK(h, hipMemsetAsync(h->lst.klo + off, 0, sizeof(int32_t) * n, h->stream));
        HIPCHK(h, hipMemsetAsync(h->lst.pstart + off, 0, sizeof(int32_t) * n, h->stream));
        HIPCHK(h, hipMemsetAsync(h->lst.pcell + off, 0, sizeof(int32_t) * n, h->stream));
    }
    k_set_thermo<<<1, 1, 0, h->stream>>>(h->thermo + TH_COUNT * slot, 0.0, 0.0);
    k_set_baro<<<1, 1, 0, h->stream>>>(h->thermo + TH_COUNT * slot, R.sp.box[0], R.sp.box[1], R.sp.box[2]);
    k_set_i64<<<1, 1, 0, h->stream>>>(h->budget + slot, kUnbounded);
    k_set_i64<<<1, 1, 0, h->stream>>>(h->steps + slot, 0);
    h->chunks.mark(R.chunk0, R.nchunks, 1);
    h->cells.mark(R.cell0, R.ncells, 1);
    h->shapes.mark(R.shape0, R.nshapes, 1);
    R.live = true;
    h->reps[slot] = R;
    place_pairs(h);
    *rid = slot;
    return upload_tables(h);
}

void release_replica(dem_system *h, int r)
{
    Replica &R = h->reps[r];
    if (!R.live) return;
    h->chunks.mark(R.chunk0, R.nchunks, 0);
    h->cells.mark(R.cell0, R.ncells, 0);
    h->shapes.mark(R.shape0, R.nshapes, 0);
    R = Replica{};
}

dem_status compute_forces(dem_system *h)
{
    const Launch L = make_launch(h);
    k_bump<<<1, 1, 0, h->stream>>>(h->lst.gflags + G_STAMP);  // a new force evaluation
    launch_rotations(L, h->stream);
    launch_pairs(L, h->stats, h->stream);
    launch_gather(L, false, h->stream);
    HIPCHK(h, hipGetLastError());
    return DEM_OK;
}

bool valid_replica(const dem_system *h, int r) { return h && r >= 0 && r < (int)h->reps.size() && h->reps[r].live; }

dem_status finish_energy(dem_system *h, int r, const double acc[12], const double th[TH_COUNT],
                         const int32_t flags[FLAG_COUNT], int64_t steps, dem_energy_out *o);

dem_status replica_energy(dem_system *h, int r, dem_energy_out *o)
{
    std::memset(o, 0, sizeof *o);
    const Replica &R = h->reps[r];
    std::vector<double> part((size_t)12 * std::max(R.nchunks, 1), 0.0);
    double th[TH_COUNT];
    int32_t flags[FLAG_COUNT];
    int64_t steps = 0;
    launch_energy_partials(make_launch(h), h->e_part, h->stream);
    HIPCHK(h, hipGetLastError());
    if (R.nchunks > 0)
        HIPCHK(h, hipMemcpyAsync(part.data(), h->e_part + (size_t)12 * R.chunk0, sizeof(double) * 12 * R.nchunks,
                                 hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(th, h->thermo + TH_COUNT * r, sizeof th, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(flags, h->lst.flags + FLAG_COUNT * r, sizeof flags, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(&steps, h->steps + r, sizeof steps, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    double acc[12] = {0};
    for (int b = 0; b < R.nchunks; ++b)
        for (int c = 0; c < 12; ++c) acc[c] += part[(size_t)12 * b + c];
    return finish_energy(h, r, acc, th, flags, steps, o);
}

// dem_energy_out of replica r from its totals of U, K_trans, K_rot and W (9),
// its thermostat words, flags and step count; latched device errors.
dem_status finish_energy(dem_system *h, int r, const double acc[12], const double th[TH_COUNT],
                         const int32_t flags[FLAG_COUNT], int64_t steps, dem_energy_out *o)
{
    const SysParams &sp = h->reps[r].sp;
    const bool npt = sp.ensemble == DEM_NPT;
    o->U = acc[0];
    o->K_trans = acc[1];
    o->K_rot = acc[2];
    for (int c = 0; c < 9; ++c) o->W[c] = acc[3 + c];
    const double K = o->K_trans + o->K_rot;
    const double g = npt ? sp.g - 1.0 : sp.g;  // the particles' degrees of freedom
    o->T = g > 0 ? 2.0 * K / g : 0.0;
    const int d = sp.dim;
    for (int a = 0; a < 3; ++a) o->box[a] = npt ? th[TH_BOXN + a] : sp.box[a];  // the box of the positions
    const double vol = d == 3 ? o->box[0] * o->box[1] * o->box[2] : o->box[0] * o->box[1];
    o->V = vol;
    const double trW = d == 3 ? o->W[0] + o->W[4] + o->W[8] : o->W[0] + o->W[4];
    o->P = (2.0 * o->K_trans + trW) / (d * vol);
    o->xi = th[TH_XI_B];
    o->eta = th[TH_ETA_B];
    o->veps = npt ? th[TH_VEPS_B] : 0.0;
    o->H = K + o->U;
    if (sp.ensemble == DEM_NVT || npt) o->H += 0.5 * sp.Qm * o->xi * o->xi + sp.g * sp.kT * o->eta;
    if (npt) o->H += 0.5 * sp.Wm * o->veps * o->veps + sp.pext * vol;
    o->step = steps;
    o->n_rebuilds = flags[FLAG_NBUILDS];
    if (flags[FLAG_NONFINITE]) return fail(h, DEM_E_NONFINITE, "non-finite position or velocity");
    if (flags[FLAG_CELLOVF])
        return fail(h, DEM_E_CAPACITY, "a cell held more than %d particles in a list build", kCellCap);
    if (flags[FLAG_MAXROW] > h->bp.cap)
        return fail(h, DEM_E_CAPACITY, "neighbour row of %d exceeds capacity %d", flags[FLAG_MAXROW], h->bp.cap);
    if (flags[FLAG_BOXSMALL])
        return fail(h, DEM_E_STATE, "the barostat shrank the box below twice the list radius %g", sp.rlist);
    return DEM_OK;
}

// replica_energy with its partials and totals in the static scratch: no
// device or host allocation.
dem_status replica_energy_noalloc(dem_system *h, int r, dem_energy_out *o)
{
    std::memset(o, 0, sizeof *o);
    const Replica &R = h->reps[r];
    if (!h->scratch) return fail(h, DEM_E_STATE, "the static scratch was not set up for this handle's device");
    if (R.nchunks > kScratchChunks)
        return fail(h, DEM_E_CAPACITY,
                    "replica %d has %d particles (%d chunks of %d); the allocation-free energy call takes at most %d "
                    "particles (%d chunks)",
                    r, R.sp.n, R.nchunks, kChunk, kScratchChunks * kChunk, kScratchChunks);
    double acc[12];
    double th[TH_COUNT];
    int32_t flags[FLAG_COUNT];
    int64_t steps = 0;
    double *total = h->scratch + kScratchTotals;
    // the totals are written whole by every call, so nothing left by an
    // earlier call reaches this one
    launch_energy_totals(make_launch(h), R.chunk0, R.nchunks, h->scratch, total, h->stream);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipMemcpyAsync(acc, total, sizeof acc, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(th, h->thermo + TH_COUNT * r, sizeof th, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(flags, h->lst.flags + FLAG_COUNT * r, sizeof flags, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(&steps, h->steps + r, sizeof steps, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return finish_energy(h, r, acc, th, flags, steps, o);
}

// The lists of replica r in their canonical form: the cell list as CSR with
// particles ascending inside each cell (from each particle's cell), rows as
// stored.  Indices are the replica's own.
dem_status copy_lists(dem_system *h, int r, int32_t *cell_start, int32_t *cell_particles, int32_t *nbr,
                      int32_t *n_nbr, int32_t *dims)
{
    if (dem_status st = sync_dynamic(h); st != DEM_OK) return st;  // an NPT replica's cells follow its box
    const Replica &R = h->reps[r];
    const size_t n = (size_t)R.sp.n, off = (size_t)R.sp.off, N = (size_t)h->bp.N;
    std::vector<int32_t> pcell(n);
    if (n) HIPCHK(h, hipMemcpyAsync(pcell.data(), h->lst.pcell + off, sizeof(int32_t) * n, hipMemcpyDeviceToHost,
                                    h->stream));
    if (nbr && n)
        HIPCHK(h, hipMemcpy2DAsync(nbr, sizeof(int32_t) * n, h->lst.nbr + off, sizeof(int32_t) * N,
                                   sizeof(int32_t) * n, (size_t)h->bp.cap, hipMemcpyDeviceToHost, h->stream));
    if (n_nbr && n)
        HIPCHK(h, hipMemcpyAsync(n_nbr, h->lst.n_nbr + off, sizeof(int32_t) * n, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    const int ncell = R.sp.ncell;
    std::vector<int32_t> start((size_t)ncell + 1, 0);
    for (size_t i = 0; i < n; ++i) start[(size_t)pcell[i] + 1] += 1;
    for (int c = 0; c < ncell; ++c) start[(size_t)c + 1] += start[c];
    if (cell_start) std::copy(start.begin(), start.end(), cell_start);
    if (cell_particles) {
        std::vector<int32_t> at(start.begin(), start.end() - 1);
        for (size_t i = 0; i < n; ++i) cell_particles[at[pcell[i]]++] = (int32_t)i;
    }
    if (nbr && n_nbr)
        for (size_t i = 0; i < n; ++i)
            for (int k = 0; k < n_nbr[i]; ++k) nbr[(size_t)k * n + i] -= (int32_t)off;
    if (dims) {
        dims[0] = R.sp.nc[0];
        dims[1] = R.sp.nc[1];
        dims[2] = R.sp.nc[2];
        dims[3] = h->bp.cap;
    }
    return DEM_OK;
}

dem_status run_steps(dem_system *h, int64_t n_steps)
{
    if (n_steps < 0) return fail(h, DEM_E_ARG, "n_steps < 0");
    if (n_steps == 0) return DEM_OK;
    for (size_t r = 0; r < h->reps.size(); ++r)
        if (h->reps[r].live && h->reps[r].sp.n == 0) k_advance_empty<<<1, 1, 0, h->stream>>>(h->budget + r, h->steps + r, n_steps);
    if (h->bp.nchunk == 0) {
        HIPCHK(h, hipGetLastError());
        return DEM_OK;
    }
    dem_status st = ensure_graph(h);
    if (st != DEM_OK) return st;
    const Launch L = make_launch(h);
    // opening half step of the first step, from the current kinetic energy
    launch_kinetic(L, h->stream);
    launch_nh_begin(L, h->stream);
    int64_t k = 0;
    for (; k + kGraphSteps <= n_steps; k += kGraphSteps) HIPCHK(h, hipGraphLaunch(h->gexec_multi, h->stream));
    for (; k < n_steps; ++k) HIPCHK(h, hipGraphLaunch(h->gexec, h->stream));
    launch_nh_end(L, h->stream);
    HIPCHK(h, hipGetLastError());
    return DEM_OK;
}

}  // namespace

extern "C" {

const char *dem_status_string(dem_status s)
{
    switch (s) {
    case DEM_OK: return "ok";
    case DEM_E_ARG: return "invalid argument";
    case DEM_E_SHAPE: return "invalid shape";
    case DEM_E_OOM: return "out of device memory";
    case DEM_E_HIP: return "HIP runtime error";
    case DEM_E_CAPACITY: return "neighbour capacity exceeded";
    case DEM_E_NONFINITE: return "non-finite state";
    case DEM_E_STATE: return "bad handle state";
    }
    return "unknown status";
}

const char *dem_last_error(dem_handle h) { return h ? h->err.c_str() : g_err.c_str(); }

size_t dem_footprint_bytes(const dem_params *p)
{
    if (!p || p->n < 0) return 0;
    const size_t n = (size_t)((std::max<int64_t>(p->n, 1) + kChunk - 1) / kChunk * kChunk);
    double Rm = 0.0, rm = 0.0;
    for (int s = 0; s < p->n_shapes && p->shapes; ++s) {
        const dem_shape_desc &d = p->shapes[s];
        for (int k = 0; k < d.n_vertices && d.vertices; ++k) {
            const double *v = d.vertices + 3 * k;
            Rm = std::max(Rm, std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
        }
        rm = std::max(rm, d.rounding_radius);
    }
    double rl = 2.0 * Rm + kWcaCut * (2.0 * rm) + p->skin;
    int cap = p->nbr_capacity > 0 ? p->nbr_capacity : auto_capacity(*p, rl);
    size_t ncell = 1;
    for (int a = 0; a < p->dim && a < 3; ++a) ncell *= (size_t)std::max(1.0, std::floor(p->box[a] / rl));
    const size_t nch = (n + kChunk - 1) / kChunk;
    const size_t maxp = n * (size_t)cap / 2;
    return sizeof(int32_t) * (n * (size_t)cap + 4 * n + ncell * (1 + kCellCap) + 8 * maxp + nch + 2 * FLAG_COUNT + G_COUNT + 2 +
                              split_words(1)) +
           sizeof(double) * (3 * n + (kKePer + 12) * nch + TH_COUNT + 2) + sizeof(unsigned long long) * ST_COUNT +
           (partrec_bytes(p->precision) + (p->precision == DEM_FP32 ? sizeof(PartRec64) : 0)) * n +
           sizeof(uint2) * kFcCells * DEM_MAX_SHAPES +
           rec_bytes(p->precision) * (size_t)cap * n + sizeof(uint32_t) * (size_t)slot_words(cap) * n + sizeof(SysParams) + 2 * DEM_MAX_SHAPES * sizeof(ShapeTab<double>) + 256;
}

dem_status dem_create_system(const dem_params *params, const dem_state_ptrs *state, const dem_output_ptrs *outputs,
                             void *hip_stream, dem_handle *out)
{
    if (out) *out = nullptr;
    if (!params || !state || !outputs || !out) return fail(nullptr, DEM_E_ARG, "null argument");
    const dem_params &p = *params;
    if (p.dim != 2 && p.dim != 3) return fail(nullptr, DEM_E_ARG, "dim must be 2 or 3");
    if (p.precision != DEM_FP64 && p.precision != DEM_FP32) return fail(nullptr, DEM_E_ARG, "bad precision");
    if (p.n < 0 || p.n > (int64_t)INT32_MAX / 64) return fail(nullptr, DEM_E_ARG, "n out of range");
    if (p.n > 0) {
        const double *req[] = {state->x, state->y, state->qw, state->qx, state->qy, state->qz, state->vx, state->vy,
                               state->vz, state->Lx, state->Ly, state->Lz, outputs->Fx, outputs->Fy, outputs->Fz,
                               outputs->Tx, outputs->Ty, outputs->Tz, outputs->U, outputs->W};
        for (const double *r : req)
            if (!r) return fail(nullptr, DEM_E_ARG, "null state or output array");
        if (!state->shape_id || !state->image || (p.dim == 3 && !state->z))
            return fail(nullptr, DEM_E_ARG, "null state array");
    }
    dem_system *h = new (std::nothrow) dem_system();
    if (!h) return fail(nullptr, DEM_E_OOM, "host allocation");
    h->batch = false;
    h->dim = p.dim;
    h->precision = p.precision;
    h->stream = (hipStream_t)hip_stream;
    auto bail = [&](dem_status s) {
        g_err = h->err;
        dem_destroy_system(h);
        return s;
    };
    Replica R;
    std::vector<ShapeTab<double>> t64;
    std::vector<ShapeTab<float>> t32;
    dem_status st = describe_replica(h, p, R, t64, t32);
    if (st != DEM_OK) return bail(st);
    h->st = {state->x, state->y, state->z, state->qw, state->qx, state->qy, state->qz, state->vx, state->vy,
             state->vz, state->Lx, state->Ly, state->Lz, state->shape_id, state->image};
    h->out = {outputs->Fx, outputs->Fy, outputs->Fz, outputs->Tx, outputs->Ty, outputs->Tz, outputs->U, outputs->W};
    h->bp.wstride = (int)p.n;
    h->bp.nstate = (int)p.n;
    if (hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(h, DEM_E_HIP, "stream creation failed"));
    if ((st = scratch_of(h)) != DEM_OK) return bail(st);
    const int nch = (int)((p.n + kChunk - 1) / kChunk);
    if ((st = alloc_core(h, nch * kChunk, R.sp.ncell + 1, p.n_shapes, 1)) != DEM_OK) return bail(st);
    h->auto_cap = p.nbr_capacity <= 0;
    if (!h->auto_cap && p.nbr_capacity > kRowMax)
        return bail(fail(h, DEM_E_ARG, "nbr_capacity %d above the limit %d", p.nbr_capacity, kRowMax));
    if ((st = alloc_nbr(h, h->auto_cap ? auto_capacity(p, R.r_list) : p.nbr_capacity)) != DEM_OK) return bail(st);
    int rid = -1;
    if ((st = place_replica(h, R, t64, t32, nullptr, &rid)) != DEM_OK) return bail(st);
    if ((st = build_lists_sync(h, LISTS_ALL)) != DEM_OK) return bail(st);
    if ((st = compute_forces(h)) != DEM_OK) return bail(st);
    if ((st = latched(h)) != DEM_OK) return bail(st);
    *out = h;
    return DEM_OK;
}

dem_status dem_batch_create(const dem_batch_params *bpar, void *hip_stream, dem_handle *out)
{
    if (out) *out = nullptr;
    if (!bpar || !out) return fail(nullptr, DEM_E_ARG, "null argument");
    const dem_batch_params &b = *bpar;
    if (b.dim != 2 && b.dim != 3) return fail(nullptr, DEM_E_ARG, "dim must be 2 or 3");
    if (b.precision != DEM_FP64 && b.precision != DEM_FP32) return fail(nullptr, DEM_E_ARG, "bad precision");
    if (b.max_replicas < 1 || b.max_replicas > 65536) return fail(nullptr, DEM_E_ARG, "max_replicas out of range");
    if (b.max_particles < 1 || b.max_particles > (int64_t)INT32_MAX / 128)
        return fail(nullptr, DEM_E_ARG, "max_particles out of range");
    if (b.max_cells < 0 || b.max_cells > (int64_t)INT32_MAX / 2 || b.max_shapes < 0 || b.nbr_capacity < 0 ||
        b.hbm_budget_bytes < 0)
        return fail(nullptr, DEM_E_ARG, "negative or oversized limit");
    dem_system *h = new (std::nothrow) dem_system();
    if (!h) return fail(nullptr, DEM_E_OOM, "host allocation");
    h->batch = true;
    h->hbm_budget = (size_t)b.hbm_budget_bytes;
    h->dim = b.dim;
    h->precision = b.precision;
    h->stream = (hipStream_t)hip_stream;
    auto bail = [&](dem_status s) {
        g_err = h->err;
        dem_destroy_system(h);
        return s;
    };
    const int Ncap = (int)((b.max_particles + kChunk - 1) / kChunk * kChunk);
    const int Ccap = b.max_cells > 0 ? (int)b.max_cells : Ncap + 2 * b.max_replicas;
    const int Scap = b.max_shapes > 0 ? b.max_shapes : DEM_MAX_SHAPES * b.max_replicas;
    dem_status st;
    if (hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(h, DEM_E_HIP, "stream creation failed"));
    if ((st = scratch_of(h)) != DEM_OK) return bail(st);
    if ((st = alloc_core(h, Ncap, Ccap, Scap, b.max_replicas)) != DEM_OK) return bail(st);
    h->auto_cap = b.nbr_capacity <= 0;
    if ((st = alloc_nbr(h, h->auto_cap ? 16 : ((b.nbr_capacity + 3) & ~3))) != DEM_OK) return bail(st);
    if ((st = upload_tables(h)) != DEM_OK) return bail(st);
    HIPCHK(h, hipStreamSynchronize(h->stream));
    *out = h;
    return DEM_OK;
}

dem_status dem_batch_add(dem_handle h, const dem_params *params, const dem_state_ptrs *state, int64_t steps,
                         int32_t *replica_id)
{
    if (replica_id) *replica_id = -1;
    if (!h || !params || !state || !replica_id) return fail(h, DEM_E_ARG, "null argument");
    if (!h->batch) return fail(h, DEM_E_STATE, "not a batch handle");
    if (steps < 0) return fail(h, DEM_E_ARG, "steps < 0");
    Replica R;
    std::vector<ShapeTab<double>> t64;
    std::vector<ShapeTab<float>> t32;
    dem_status st = describe_replica(h, *params, R, t64, t32);
    if (st != DEM_OK) return st;
    const size_t slots = (size_t)((params->n + kChunk - 1) / kChunk) * kChunk;
    if (slots > (size_t)h->Ncap) return fail(h, DEM_E_OOM, "replica larger than the batch");
    // admission by footprint: its lists, cells and scratch, plus its state
    // and outputs in the batch's arrays
    R.bytes = dem_footprint_bytes(params) + slots * (16 * sizeof(double) + 4 * sizeof(int32_t));
    if (h->hbm_budget > 0 && h->hbm_used + R.bytes > h->hbm_budget)
        return fail(h, DEM_E_OOM, "replica of %zu bytes does not fit the admission budget (%zu of %zu bytes in use)",
                    R.bytes, h->hbm_used, h->hbm_budget);
    const int want = h->auto_cap ? auto_capacity(*params, R.r_list) : h->bp.cap;
    int rid = -1;
    if ((st = place_replica(h, R, t64, t32, state, &rid)) != DEM_OK) return st;
    h->hbm_used += R.bytes;
    if (want > h->bp.cap) {
        if ((st = alloc_nbr(h, want)) != DEM_OK) return st;
    }
    if ((st = build_lists_sync(h, rid)) != DEM_OK) return st;
    if ((st = compute_forces(h)) != DEM_OK) return st;
    if (steps > 0) k_set_i64<<<1, 1, 0, h->stream>>>(h->budget + rid, steps);
    HIPCHK(h, hipGetLastError());
    *replica_id = rid;
    return DEM_OK;
}

dem_status dem_batch_remove(dem_handle h, int32_t rid)
{
    if (!h || !h->batch) return fail(h, DEM_E_ARG, "not a batch handle");
    if (!valid_replica(h, rid)) return fail(h, DEM_E_ARG, "no replica %d", rid);
    k_retire_flags<<<1, 1, 0, h->stream>>>(h->lst.flags + FLAG_COUNT * rid, h->lst.gflags);
    h->hbm_used -= std::min(h->hbm_used, h->reps[rid].bytes);
    release_replica(h, rid);
    place_pairs(h);
    dem_status st = upload_tables(h);
    if (st != DEM_OK) return st;
    launch_lists(make_launch(h), LISTS_PLAN, h->stream);  // the tile plan drops the replica
    HIPCHK(h, hipGetLastError());
    return DEM_OK;
}

dem_status dem_batch_read(dem_handle h, int32_t rid, const dem_state_ptrs *state, const dem_output_ptrs *outputs)
{
    if (!h || !h->batch) return fail(h, DEM_E_ARG, "not a batch handle");
    if (!valid_replica(h, rid)) return fail(h, DEM_E_ARG, "no replica %d", rid);
    const Replica &R = h->reps[rid];
    const size_t n = (size_t)R.sp.n, off = (size_t)R.sp.off;
    if (n == 0) return DEM_OK;
    if (state) {
        double *to[] = {state->x, state->y, state->z, state->qw, state->qx, state->qy, state->qz,
                        state->vx, state->vy, state->vz, state->Lx, state->Ly, state->Lz};
        const double *from[] = {h->st.x, h->st.y, h->st.z, h->st.qw, h->st.qx, h->st.qy, h->st.qz,
                                h->st.vx, h->st.vy, h->st.vz, h->st.Lx, h->st.Ly, h->st.Lz};
        for (int k = 0; k < 13; ++k)
            if (to[k])
                HIPCHK(h, hipMemcpyAsync(to[k], from[k] + off, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
        if (state->shape_id)
            HIPCHK(h, hipMemcpyAsync(state->shape_id, h->st.sid + off, sizeof(int32_t) * n, hipMemcpyDeviceToDevice,
                                     h->stream));
        if (state->image)
            HIPCHK(h, hipMemcpyAsync(state->image, h->st.image + 3 * off, sizeof(int32_t) * 3 * n,
                                     hipMemcpyDeviceToDevice, h->stream));
    }
    if (outputs) {
        double *to[] = {outputs->Fx, outputs->Fy, outputs->Fz, outputs->Tx, outputs->Ty, outputs->Tz, outputs->U};
        const double *from[] = {h->out.Fx, h->out.Fy, h->out.Fz, h->out.Tx, h->out.Ty, h->out.Tz, h->out.U};
        for (int k = 0; k < 7; ++k)
            if (to[k])
                HIPCHK(h, hipMemcpyAsync(to[k], from[k] + off, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
        if (outputs->W)
            HIPCHK(h, hipMemcpy2DAsync(outputs->W, sizeof(double) * n, h->out.W + off, sizeof(double) * h->bp.wstride,
                                       sizeof(double) * n, 9, hipMemcpyDeviceToDevice, h->stream));
    }
    return DEM_OK;
}

dem_status dem_batch_set_steps(dem_handle h, int32_t rid, int64_t steps)
{
    if (!h || !h->batch) return fail(h, DEM_E_ARG, "not a batch handle");
    if (!valid_replica(h, rid)) return fail(h, DEM_E_ARG, "no replica %d", rid);
    k_set_i64<<<1, 1, 0, h->stream>>>(h->budget + rid, steps > 0 ? steps : 0);
    HIPCHK(h, hipGetLastError());
    return DEM_OK;
}

dem_status dem_batch_progress(dem_handle h, int64_t *steps_left, int64_t *steps_done, int32_t count)
{
    if (!h || count < 0) return fail(h, DEM_E_ARG, "bad argument");
    const int n = std::min<int>(count, (int)h->reps.size());
    if (n > 0 && steps_left)
        HIPCHK(h, hipMemcpyAsync(steps_left, h->budget, sizeof(int64_t) * n, hipMemcpyDeviceToHost, h->stream));
    if (n > 0 && steps_done)
        HIPCHK(h, hipMemcpyAsync(steps_done, h->steps, sizeof(int64_t) * n, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int r = 0; r < n; ++r)
        if (!h->reps[r].live) {
            if (steps_left) steps_left[r] = -1;
            if (steps_done) steps_done[r] = -1;
        }
    return latched(h);
}

dem_status dem_batch_info(dem_handle h, int64_t *out)
{
    if (!h || !out) return fail(h, DEM_E_ARG, "null argument");
    int live = 0;
    for (const Replica &R : h->reps) live += R.live ? 1 : 0;
    int run = 0, best = 0;
    for (int k = 0; k < h->chunks.size(); ++k) {
        run = h->chunks.used[k] ? 0 : run + 1;
        best = std::max(best, run);
    }
    out[0] = live;
    out[1] = (int64_t)h->reps.size();
    out[2] = (int64_t)h->chunks.free_slots() * kChunk;
    out[3] = (int64_t)best * kChunk;
    out[4] = h->cells.free_slots();
    out[5] = h->shapes.free_slots();
    out[6] = h->bp.cap;
    out[7] = h->Ncap;
    out[8] = (int64_t)h->hbm_used;
    out[9] = (int64_t)h->hbm_budget;
    return DEM_OK;
}

dem_status dem_destroy_system(dem_handle h)
{
    if (!h) return DEM_E_ARG;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    free_all(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    delete h;
    return DEM_OK;
}

dem_status dem_build_celllist(dem_handle h)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    return build_lists_sync(h, LISTS_ALL);
}

dem_status dem_compute_forces(dem_handle h)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    return compute_forces(h);
}

dem_status dem_step(dem_handle h, int64_t n_steps)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    return run_steps(h, n_steps);
}

dem_status dem_sync(dem_handle h)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    HIPCHK(h, hipGetLastError());
    return latched(h);
}

dem_status dem_energy(dem_handle h, dem_energy_out *o)
{
    if (!h || !o) return fail(h, DEM_E_ARG, "null argument");
    if (!valid_replica(h, 0)) return fail(h, DEM_E_ARG, "no replica 0");
    return replica_energy(h, 0, o);
}

dem_status dem_replica_energy(dem_handle h, int32_t rid, dem_energy_out *o)
{
    if (!h || !o) return fail(h, DEM_E_ARG, "null argument");
    if (!valid_replica(h, rid)) return fail(h, DEM_E_ARG, "no replica %d", rid);
    return replica_energy(h, rid, o);
}

dem_status dem_replica_energy_noalloc(dem_handle h, int32_t rid, dem_energy_out *o)
{
    if (!o) return fail(h, DEM_E_ARG, "null argument");
    if (!valid_replica(h, rid)) return fail(h, DEM_E_ARG, "no live replica %d", rid);
    return replica_energy_noalloc(h, rid, o);
}

dem_status dem_set_thermostat(dem_handle h, double xi, double eta)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    if (!valid_replica(h, 0)) return fail(h, DEM_E_ARG, "no replica 0");
    k_set_thermo<<<1, 1, 0, h->stream>>>(h->thermo, xi, eta);
    HIPCHK(h, hipGetLastError());
    return DEM_OK;
}

dem_status dem_set_barostat(dem_handle h, double veps)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    if (!valid_replica(h, 0) || h->reps[0].sp.ensemble != DEM_NPT) return fail(h, DEM_E_ARG, "not an NPT system");
    if (!std::isfinite(veps)) return fail(h, DEM_E_ARG, "non-finite v_eps");
    k_set_veps<<<1, 1, 0, h->stream>>>(h->thermo, veps);
    HIPCHK(h, hipGetLastError());
    return DEM_OK;
}

dem_status dem_copy_lists(dem_handle h, int32_t *cell_start, int32_t *cell_particles, int32_t *nbr, int32_t *n_nbr,
                          int32_t *dims)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    if (!valid_replica(h, 0)) return fail(h, DEM_E_ARG, "no replica 0");
    return copy_lists(h, 0, cell_start, cell_particles, nbr, n_nbr, dims);
}

dem_status dem_replica_lists(dem_handle h, int32_t rid, int32_t *cell_start, int32_t *cell_particles, int32_t *nbr,
                             int32_t *n_nbr, int32_t *dims)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    if (!valid_replica(h, rid)) return fail(h, DEM_E_ARG, "no replica %d", rid);
    return copy_lists(h, rid, cell_start, cell_particles, nbr, n_nbr, dims);
}

dem_status dem_list_info(dem_handle h, double *r_list, int32_t *n_cells, int32_t *capacity)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    if (!valid_replica(h, 0)) return fail(h, DEM_E_ARG, "no replica 0");
    if (r_list) *r_list = h->reps[0].r_list;
    if (n_cells) *n_cells = h->reps[0].sp.ncell;
    if (capacity) *capacity = h->bp.cap;
    return DEM_OK;
}

dem_status dem_force_stats(dem_handle h, int64_t *out, int32_t reset)
{
    if (!h || !out) return fail(h, DEM_E_ARG, "null argument");
    unsigned long long v[ST_COUNT];
    HIPCHK(h, hipMemcpyAsync(v, h->stats, sizeof v, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int k = 0; k < ST_COUNT; ++k) out[k] = (int64_t)v[k];
    if (reset) HIPCHK(h, hipMemsetAsync(h->stats, 0, sizeof v, h->stream));
    return DEM_OK;
}

dem_status dem_set_counting(dem_handle h, int32_t on)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    if ((on != 0) != h->counting) {
        h->counting = on != 0;
        drop_graph(h);
    }
    return DEM_OK;
}

dem_status dem_time_forces(dem_handle h, int32_t reps, double *mean_ms)
{
    if (!h || !mean_ms || reps < 1) return fail(h, DEM_E_ARG, "bad argument");
    // The launches are captured in one graph, so they run back to back as
    // in a step graph and the mean is the kernel's own duration (separate
    // launches would add the host-side gap between them).
    const Launch L = make_launch(h);
    HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int r = 0; r < reps; ++r) launch_pairs(L, nullptr, h->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    if (e != hipSuccess || !g) return fail(h, DEM_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.0f;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipGraphLaunch(x, h->stream);  // warm
    if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
    if (e == hipSuccess) e = hipGraphLaunch(x, h->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (x) (void)hipGraphExecDestroy(x);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(h, DEM_E_HIP, "force timing failed: %s", hipGetErrorString(e));
    *mean_ms = (double)ms / reps;
    return DEM_OK;
}

dem_status dem_batch_step(dem_handle h, int64_t n_steps) { return dem_step(h, n_steps); }

dem_status dem_get_outputs(dem_handle h, dem_output_view *o)
{
    if (!h || !o) return fail(h, DEM_E_ARG, "null argument");
    o->Fx = h->out.Fx;
    o->Fy = h->out.Fy;
    o->Fz = h->out.Fz;
    o->Tx = h->out.Tx;
    o->Ty = h->out.Ty;
    o->Tz = h->out.Tz;
    o->U = h->out.U;
    o->W = h->out.W;
    o->w_stride = h->bp.wstride;
    o->nbr = h->lst.nbr;
    o->n_nbr = h->lst.n_nbr;
    o->nbr_stride = h->bp.N;
    o->capacity = h->bp.cap;
    return DEM_OK;
}

// Checkpoint layout: this header, then x, y, z, qw, qx, qy, qz, vx, vy, vz,
// Lx, Ly, Lz (n doubles each; z is zero in 2D), shape id (n int32) and
// image (3n int32).
struct CheckpointHeader {
    char magic[8];
    int32_t version, dim;
    int64_t n, step, n_rebuilds;
    double thermo[TH_COUNT];
};
constexpr char kCheckpointMagic[8] = {'D', 'E', 'M', 'C', 'K', 'P', 'T', '1'};

size_t dem_state_bytes(dem_handle h)
{
    if (!h || h->batch || !valid_replica(h, 0)) return 0;
    const size_t n = (size_t)h->reps[0].sp.n;
    return sizeof(CheckpointHeader) + n * (13 * sizeof(double) + 4 * sizeof(int32_t));
}

dem_status dem_get_state(dem_handle h, void *host_buf, size_t bytes)
{
    if (!h || !host_buf) return fail(h, DEM_E_ARG, "null argument");
    if (h->batch || !valid_replica(h, 0)) return fail(h, DEM_E_ARG, "checkpoints are for single systems");
    const size_t need = dem_state_bytes(h);
    if (bytes < need) return fail(h, DEM_E_ARG, "checkpoint buffer of %zu bytes, %zu needed", bytes, need);
    const size_t n = (size_t)h->reps[0].sp.n;
    unsigned char *b = static_cast<unsigned char *>(host_buf);
    CheckpointHeader hd{};
    std::memcpy(hd.magic, kCheckpointMagic, 8);
    hd.version = 2;
    hd.dim = h->dim;
    hd.n = (int64_t)n;
    int32_t nb = 0;
    HIPCHK(h, hipMemcpyAsync(hd.thermo, h->thermo, sizeof hd.thermo, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(&hd.step, h->steps, sizeof hd.step, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(&nb, h->lst.flags + FLAG_NBUILDS, sizeof nb, hipMemcpyDeviceToHost, h->stream));
    double *dst = reinterpret_cast<double *>(b + sizeof hd);
    double *const cols[13] = {h->st.x, h->st.y, h->st.z, h->st.qw, h->st.qx, h->st.qy, h->st.qz,
                              h->st.vx, h->st.vy, h->st.vz, h->st.Lx, h->st.Ly, h->st.Lz};
    for (int c = 0; c < 13; ++c) {
        if (cols[c] && n) HIPCHK(h, hipMemcpyAsync(dst + c * n, cols[c], sizeof(double) * n, hipMemcpyDeviceToHost, h->stream));
        else std::memset(dst + c * n, 0, sizeof(double) * n);
    }
    int32_t *idst = reinterpret_cast<int32_t *>(dst + 13 * n);
    if (n) {
        HIPCHK(h, hipMemcpyAsync(idst, h->st.sid, sizeof(int32_t) * n, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipMemcpyAsync(idst + n, h->st.image, sizeof(int32_t) * 3 * n, hipMemcpyDeviceToHost, h->stream));
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    hd.n_rebuilds = nb;
    std::memcpy(b, &hd, sizeof hd);
    return DEM_OK;
}

dem_status dem_set_state(dem_handle h, const void *host_buf, size_t bytes)
{
    if (!h || !host_buf) return fail(h, DEM_E_ARG, "null argument");
    if (h->batch || !valid_replica(h, 0)) return fail(h, DEM_E_ARG, "checkpoints are for single systems");
    const size_t n = (size_t)h->reps[0].sp.n;
    if (bytes < sizeof(CheckpointHeader)) return fail(h, DEM_E_ARG, "checkpoint too short");
    CheckpointHeader hd;
    std::memcpy(&hd, host_buf, sizeof hd);
    if (std::memcmp(hd.magic, kCheckpointMagic, 8) != 0 || hd.version != 2)
        return fail(h, DEM_E_ARG, "not a checkpoint of this library");
    if (hd.dim != h->dim || hd.n != (int64_t)n) return fail(h, DEM_E_ARG, "checkpoint of another system");
    if (bytes < dem_state_bytes(h)) return fail(h, DEM_E_ARG, "checkpoint too short");
    const unsigned char *b = static_cast<const unsigned char *>(host_buf);
    const double *src = reinterpret_cast<const double *>(b + sizeof hd);
    double *const cols[13] = {h->st.x, h->st.y, h->st.z, h->st.qw, h->st.qx, h->st.qy, h->st.qz,
                              h->st.vx, h->st.vy, h->st.vz, h->st.Lx, h->st.Ly, h->st.Lz};
    for (int c = 0; c < 13; ++c)
        if (cols[c] && n) HIPCHK(h, hipMemcpyAsync(cols[c], src + c * n, sizeof(double) * n, hipMemcpyHostToDevice, h->stream));
    const int32_t *isrc = reinterpret_cast<const int32_t *>(src + 13 * n);
    if (n) {
        HIPCHK(h, hipMemcpyAsync(h->st.sid, isrc, sizeof(int32_t) * n, hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(h->st.image, isrc + n, sizeof(int32_t) * 3 * n, hipMemcpyHostToDevice, h->stream));
    }
    HIPCHK(h, hipMemcpyAsync(h->thermo, hd.thermo, sizeof hd.thermo, hipMemcpyHostToDevice, h->stream));
    k_box_restore<<<1, 1, 0, h->stream>>>(h->d_reps, 0, h->lst, h->thermo);  // the box of the restored positions
    k_set_i64<<<1, 1, 0, h->stream>>>(h->steps, hd.step);
    // latched device errors belong to the state being replaced
    for (int w : {FLAG_NONFINITE, FLAG_MAXROW, FLAG_CELLOVF, FLAG_BOXSMALL})
        k_set_i32<<<1, 1, 0, h->stream>>>(h->lst.flags + w, 0);
    HIPCHK(h, hipStreamSynchronize(h->stream));  // the host buffer may be freed on return
    dem_status st = build_lists_sync(h, LISTS_ALL);
    if (st == DEM_OK) st = compute_forces(h);
    if (st != DEM_OK) return st;
    k_set_i32<<<1, 1, 0, h->stream>>>(h->lst.flags + FLAG_NBUILDS, (int32_t)hd.n_rebuilds);
    HIPCHK(h, hipGetLastError());
    return latched(h);
}

dem_status dem_set_pair_shape(dem_handle h, int32_t lanes_per_pair, int32_t grid_factor, int32_t waves_per_simd,
                              int32_t sep_lanes, int32_t split)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    if ((lanes_per_pair != 8 && lanes_per_pair != 16) || grid_factor < 1 || grid_factor > 4 ||
        (waves_per_simd != 2 && waves_per_simd != 3) || (sep_lanes != 4 && sep_lanes != 16) ||
        (sep_lanes == 16 && lanes_per_pair != 16) || (split != 0 && split != 1) || (split == 1 && sep_lanes != 4))
        return fail(h, DEM_E_ARG,
                    "pair shape: %d lanes per pair (8 or 16), grid factor %d (1 to 4), %d waves per SIMD (2 or 3), "
                    "%d separation lanes (4, or 16 with 16 lanes per pair), split %d (0, or 1 with 4 separation lanes)",
                    lanes_per_pair, grid_factor, waves_per_simd, sep_lanes, split);
    if (lanes_per_pair == h->pair_lanes && grid_factor == h->pair_grid && waves_per_simd == h->pair_waves &&
        sep_lanes == h->pair_sep && split == h->pair_split)
        return DEM_OK;
    h->pair_lanes = lanes_per_pair;
    h->pair_grid = grid_factor;
    h->pair_waves = waves_per_simd;
    h->pair_sep = sep_lanes;
    h->pair_split = split;
    refresh_batch(h);
    launch_lists(make_launch(h), LISTS_PLAN, h->stream);  // tiles of the new size
    HIPCHK(h, hipGetLastError());
    drop_graph(h);
    return DEM_OK;
}

dem_status dem_set_feature_cells(dem_handle h, int32_t on)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    if (on != 0 && on != 1) return fail(h, DEM_E_ARG, "feature cells: %d (0 or 1)", on);
    if (on == h->feature_cells) return DEM_OK;
    h->feature_cells = on;
    refresh_batch(h);
    drop_graph(h);
    return DEM_OK;
}

dem_status dem_tune_pairs(dem_handle h, int32_t reps, int32_t *shape, double *mean_ms)
{
    if (!h || reps < 1) return fail(h, DEM_E_ARG, "bad argument");
    static const int kShapes[DEM_PAIR_SHAPES][5] = {
        {16, 1, 2, 4, 0},  {8, 1, 2, 4, 0},  {16, 2, 2, 4, 0},  {8, 2, 2, 4, 0},  {16, 1, 3, 4, 0},  {8, 1, 3, 4, 0},
        {16, 2, 3, 4, 0},  {8, 2, 3, 4, 0},  {16, 1, 2, 16, 0}, {16, 2, 2, 16, 0}, {16, 1, 3, 16, 0}, {16, 2, 3, 16, 0},
        {16, 1, 2, 4, 1},  {8, 1, 2, 4, 1},  {16, 1, 3, 4, 1},  {8, 1, 3, 4, 1}};
    double best = 0.0;
    int pick = 0;
    for (int k = 0; k < DEM_PAIR_SHAPES; ++k) {
        dem_status st = dem_set_pair_shape(h, kShapes[k][0], kShapes[k][1], kShapes[k][2], kShapes[k][3], kShapes[k][4]);
        double ms = 0.0;
        if (st == DEM_OK) st = dem_time_forces(h, reps, &ms);
        if (st != DEM_OK) return st;
        if (mean_ms) mean_ms[k] = ms;
        if (k == 0 || ms < best) {
            best = ms;
            pick = k;
        }
    }
    dem_status st =
        dem_set_pair_shape(h, kShapes[pick][0], kShapes[pick][1], kShapes[pick][2], kShapes[pick][3], kShapes[pick][4]);
    if (st != DEM_OK) return st;
    if (shape)
        for (int a = 0; a < 5; ++a) shape[a] = kShapes[pick][a];
    return DEM_OK;
}

}  // extern "C"

// libdem host runtime: the C ABI of dem.h.
//
// A handle owns the device copies of the shape tables (FP64 and FP32), the
// cell and neighbour lists, flags, reduction scratch and one captured graph
// of a whole time step, which dem_step replays.  State and outputs are the
// caller's device arrays.  Every launch goes to the caller's stream; graphs
// are recorded on a private stream and launched on the caller's.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dem_internal.h"

using namespace dem;

struct dem_system {
    dem_params prm{};
    SysParams sp{};
    StatePtrs st{};
    OutPtrs out{};
    ListPtrs lst{};
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    void *tab64 = nullptr, *tab32 = nullptr;
    void *rot = nullptr;          // [9][n] in the force precision
    void *rec = nullptr;          // [max_pairs][kRec] in the force precision
    double *ke_part = nullptr;    // [2 * nblk]
    double *e_part = nullptr;     // [12 * nblk]
    double *thermo = nullptr;     // [TH_COUNT]
    unsigned long long *stats = nullptr;
    int nblk = 0;
    bool auto_cap = true;
    bool counting = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int64_t step = 0;
    double r_list = 0.0;
    std::string err;
};

namespace {

std::string g_err;

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

#define HIPCHK(h, call)                                                                            \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return fail(h, DEM_E_HIP, "%s: %s", #call, hipGetErrorString(e_));  \
    } while (0)

__global__ void k_set_int(int32_t *p, int32_t v) { *p = v; }
__global__ void k_end_build(int32_t *flags)
{
    if (flags[FLAG_REBUILD] != 0) flags[FLAG_NBUILDS] += 1;
    flags[FLAG_REBUILD] = 0;
}
__global__ void k_set_thermo(double *th, double xi, double eta)
{
    th[TH_XI] = th[TH_XI_B] = xi;
    th[TH_ETA] = th[TH_ETA_B] = eta;
    th[TH_SCALE] = th[TH_SCALE_B] = 1.0;
}

struct HostVec {
    double x, y, z;
};
inline HostVec hsub(HostVec a, HostVec b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline HostVec hcross(HostVec a, HostVec b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double hdot(HostVec a, HostVec b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// Validates one shape and fills the FP64 table.
dem_status build_table(dem_system *h, int idx, const dem_shape_desc &d, int dim, ShapeTab<double> &T)
{
    std::memset(&T, 0, sizeof T);
    if (d.dim != dim) return fail(h, DEM_E_SHAPE, "shape %d: dim %d differs from system dim %d", idx, d.dim, dim);
    if (d.n_vertices < (dim == 3 ? 4 : 3) || d.n_vertices > DEM_MAX_VERTS)
        return fail(h, DEM_E_SHAPE, "shape %d: %d vertices (limit %d)", idx, d.n_vertices, DEM_MAX_VERTS);
    if (d.n_edges < 3 || d.n_edges > DEM_MAX_EDGES)
        return fail(h, DEM_E_SHAPE, "shape %d: %d edges (limit %d)", idx, d.n_edges, DEM_MAX_EDGES);
    if (dim == 3 && (d.n_faces < 4 || d.n_faces > DEM_MAX_FACES))
        return fail(h, DEM_E_SHAPE, "shape %d: %d faces (limit %d)", idx, d.n_faces, DEM_MAX_FACES);
    if (!d.vertices || !d.edges || (dim == 3 && (!d.face_offsets || !d.face_vertices)))
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
    if (dim == 3) {
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
    return DEM_OK;
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
}

int auto_capacity(const dem_params &p, double rl)
{
    double vol = p.dim == 3 ? p.box[0] * p.box[1] * p.box[2] : p.box[0] * p.box[1];
    double dens = vol > 0.0 ? (double)p.n / vol : 0.0;
    double expect = p.dim == 3 ? dens * 4.0 / 3.0 * M_PI * rl * rl * rl : dens * M_PI * rl * rl;
    int cap = (int)std::ceil(1.8 * expect) + 16;
    cap = (cap + 3) & ~3;
    return std::max(16, std::min(cap, (int)std::max<int64_t>(p.n, 16)));
}

void free_lists(dem_system *h)
{
    (void)hipFree(h->lst.cell_count);
    (void)hipFree(h->lst.cell_start);
    (void)hipFree(h->lst.cell_particles);
    (void)hipFree(h->lst.pcell);
    (void)hipFree(h->lst.nbr);
    (void)hipFree(h->lst.n_nbr);
    (void)hipFree(h->lst.xlast);
    (void)hipFree(h->lst.klo);
    (void)hipFree(h->lst.pstart);
    (void)hipFree(h->lst.pairs);
    (void)hipFree(h->rec);
    (void)hipFree(h->rot);
    int32_t *flags = h->lst.flags;  // freed with the handle
    h->lst = ListPtrs{};
    h->lst.flags = flags;
    h->rec = h->rot = nullptr;
}

void drop_graph(dem_system *h)
{
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
}

size_t force_word(const dem_system *h) { return h->prm.precision == DEM_FP32 ? sizeof(float) : sizeof(double); }

// Row storage and everything sized by the row capacity: slot -> pair map,
// pair arrays and pair records.
dem_status alloc_nbr(dem_system *h, int cap)
{
    (void)hipFree(h->lst.nbr);
    (void)hipFree(h->lst.pairs);
    (void)hipFree(h->rec);
    h->lst.nbr = nullptr;
    h->lst.pairs = nullptr;
    h->rec = nullptr;
    const size_t n = (size_t)std::max(h->sp.n, 1);
    const size_t maxp = n * (size_t)cap / 2 + 64;
    if (maxp > (size_t)INT32_MAX) return fail(h, DEM_E_ARG, "pair capacity overflows int32");
    if (hipMalloc(&h->lst.nbr, sizeof(int32_t) * (size_t)cap * n) != hipSuccess ||
        hipMalloc(&h->lst.pairs, sizeof(int4) * maxp) != hipSuccess ||
        hipMalloc(&h->rec, force_word(h) * kRec * (size_t)cap * n) != hipSuccess)
        return fail(h, DEM_E_OOM, "neighbour list of %d x %zu entries", cap, n);
    h->sp.cap = cap;
    h->sp.max_pairs = (int)maxp;
    // grid-stride pair kernel: enough waves to fill the chip, no more than the pairs need
    const size_t want = (maxp + 15) / 16;  // four waves per block, four pairs per wave
    h->sp.pair_blocks = (int)std::max<size_t>(8, std::min<size_t>(want, 2048));
    drop_graph(h);
    return DEM_OK;
}

ForcePtrs force_ptrs(const dem_system *h)
{
    ForcePtrs f;
    f.rot = h->rot;
    f.rec = h->rec;
    f.tab = h->prm.precision == DEM_FP32 ? h->tab32 : h->tab64;
    f.tab64 = h->tab64;
    return f;
}

dem_status latched(dem_system *h)
{
    int32_t flags[FLAG_COUNT];
    HIPCHK(h, hipMemcpyAsync(flags, h->lst.flags, sizeof flags, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (flags[FLAG_NONFINITE]) return fail(h, DEM_E_NONFINITE, "non-finite position or velocity");
    if (flags[FLAG_MAXROW] > h->sp.cap)
        return fail(h, DEM_E_CAPACITY, "neighbour row of %d exceeds capacity %d", flags[FLAG_MAXROW], h->sp.cap);
    return DEM_OK;
}

void enqueue_step(dem_system *h, hipStream_t s)
{
    const ForcePtrs f = force_ptrs(h);
    launch_kick_drift(h->sp, h->st, h->out, h->lst, h->thermo, h->rot, h->prm.precision, s);
    launch_build_lists(h->sp, h->st, h->lst, s);
    launch_pairs(h->sp, h->st, h->lst, f, h->prm.precision, h->counting ? h->stats : nullptr, s);
    launch_gather(h->sp, h->st, h->out, h->lst, f, h->prm.precision, true, h->ke_part, h->thermo, s);
}

dem_status ensure_graph(dem_system *h)
{
    if (h->gexec) return DEM_OK;
    HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    enqueue_step(h, h->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    if (e != hipSuccess || !g) return fail(h, DEM_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    h->graph = g;
    HIPCHK(h, hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
    return DEM_OK;
}

dem_status build_lists_sync(dem_system *h)
{
    for (int attempt = 0; attempt < 4; ++attempt) {
        k_set_int<<<1, 1, 0, h->stream>>>(h->lst.flags + FLAG_REBUILD, 1);
        k_set_int<<<1, 1, 0, h->stream>>>(h->lst.flags + FLAG_MAXROW, 0);
        launch_build_lists(h->sp, h->st, h->lst, h->stream);
        HIPCHK(h, hipGetLastError());
        int32_t maxrow = 0;
        HIPCHK(h, hipMemcpyAsync(&maxrow, h->lst.flags + FLAG_MAXROW, sizeof maxrow, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        if (maxrow <= h->sp.cap) return DEM_OK;
        if (!h->auto_cap)
            return fail(h, DEM_E_CAPACITY, "neighbour row of %d exceeds capacity %d", maxrow, h->sp.cap);
        dem_status st = alloc_nbr(h, ((maxrow * 5) / 4 + 8 + 3) & ~3);
        if (st != DEM_OK) return st;
    }
    return fail(h, DEM_E_CAPACITY, "neighbour capacity did not converge");
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
    const size_t n = (size_t)std::max<int64_t>(p->n, 1);
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
    size_t nblk = (n + kBlock - 1) / kBlock;
    const size_t w = p->precision == DEM_FP32 ? sizeof(float) : sizeof(double);
    const size_t maxp = n * (size_t)cap / 2 + 64;
    return sizeof(int32_t) * (n * (size_t)cap + 6 * n + 2 * ncell + 2 + 4 * maxp) +
           sizeof(double) * (3 * n + 14 * nblk + TH_COUNT) + w * (16 * n + kRec * (size_t)cap * n) +
           2 * DEM_MAX_SHAPES * sizeof(ShapeTab<double>) + 256;
}

dem_status dem_create_system(const dem_params *params, const dem_state_ptrs *state, const dem_output_ptrs *outputs,
                             void *hip_stream, dem_handle *out)
{
    if (out) *out = nullptr;
    if (!params || !state || !outputs || !out) return fail(nullptr, DEM_E_ARG, "null argument");
    const dem_params &p = *params;
    if (p.dim != 2 && p.dim != 3) return fail(nullptr, DEM_E_ARG, "dim must be 2 or 3");
    if (p.n < 0 || p.n > (int64_t)INT32_MAX / 64) return fail(nullptr, DEM_E_ARG, "n out of range");
    if (p.n_shapes < 1 || p.n_shapes > DEM_MAX_SHAPES || !p.shapes)
        return fail(nullptr, DEM_E_ARG, "n_shapes must be 1..%d", DEM_MAX_SHAPES);
    if (p.ensemble != DEM_NVE && p.ensemble != DEM_NVT) return fail(nullptr, DEM_E_ARG, "bad ensemble");
    if (p.precision != DEM_FP64 && p.precision != DEM_FP32) return fail(nullptr, DEM_E_ARG, "bad precision");
    if (p.list_mode != DEM_LISTS_AUTO && p.list_mode != DEM_LISTS_MULTI) return fail(nullptr, DEM_E_ARG, "bad list_mode");
    if (!(p.dt > 0.0) || !(p.skin >= 0.0) || !(p.rebuild_frac > 0.0) || !(p.epsilon > 0.0) || !(p.parallel_sin2 >= 0.0))
        return fail(nullptr, DEM_E_ARG, "dt, epsilon, rebuild_frac must be > 0; skin, parallel_sin2 >= 0");
    if (p.ensemble == DEM_NVT && (!(p.kT > 0.0) || !(p.tau_T > 0.0)))
        return fail(nullptr, DEM_E_ARG, "NVT needs kT > 0 and tau_T > 0");
    for (int a = 0; a < p.dim; ++a)
        if (!(p.box[a] > 0.0)) return fail(nullptr, DEM_E_ARG, "box must be positive");
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
    h->prm = p;
    h->prm.shapes = nullptr;
    h->stream = (hipStream_t)hip_stream;
    auto bail = [&](dem_status s) {
        dem_destroy_system(h);
        return s;
    };

    std::vector<ShapeTab<double>> t64(p.n_shapes);
    std::vector<ShapeTab<float>> t32(p.n_shapes);
    double Rmax = 0.0, rmax = 0.0;
    SysParams &sp = h->sp;
    std::memset(&sp, 0, sizeof sp);
    for (int s = 0; s < p.n_shapes; ++s) {
        dem_status st = build_table(h, s, p.shapes[s], p.dim, t64[s]);
        if (st != DEM_OK) {
            g_err = h->err;
            return bail(st);
        }
        to_float(t64[s], t32[s]);
        sp.mass[s] = p.shapes[s].mass;
        for (int a = 0; a < 3; ++a) sp.inertia[s][a] = (p.dim == 2 && a < 2) ? 0.0 : p.shapes[s].inertia[a];
        sp.R[s] = t64[s].R;
        sp.rad[s] = p.shapes[s].rounding_radius;
        Rmax = std::max(Rmax, t64[s].R);
        rmax = std::max(rmax, p.shapes[s].rounding_radius);
    }
    // r_list = 2 R_max + 2^(1/6) sigma_max + skin
    const double rl = 2.0 * Rmax + kWcaCut * (2.0 * rmax) + p.skin;
    h->r_list = rl;
    sp.n = (int)p.n;
    sp.dim = p.dim;
    sp.n_shapes = p.n_shapes;
    sp.ensemble = p.ensemble;
    sp.use_cells = 1;
    sp.force_multi_kernel_lists = p.list_mode == DEM_LISTS_MULTI ? 1 : 0;
    for (int a = 0; a < 3; ++a) {
        sp.box[a] = (a < p.dim) ? p.box[a] : 1.0;
        if (a < p.dim) {
            if (p.box[a] < 2.0 * rl)
                return bail(fail(h, DEM_E_ARG, "box %g on axis %d is below 2 r_list = %g", p.box[a], a, 2.0 * rl));
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
    sp.Qm = sp.g * p.kT * p.tau_T * p.tau_T;

    h->st = {state->x, state->y, p.dim == 3 ? state->z : nullptr, state->qw, state->qx, state->qy, state->qz,
             state->vx, state->vy, state->vz, state->Lx, state->Ly, state->Lz, state->shape_id, state->image};
    if (p.dim == 2) h->st.z = state->z;  // may be null; never read in 2D
    h->out = {outputs->Fx, outputs->Fy, outputs->Fz, outputs->Tx, outputs->Ty, outputs->Tz, outputs->U, outputs->W};

    const size_t n = (size_t)std::max(sp.n, 1);
    h->nblk = (int)((n + kBlock - 1) / kBlock);
    const int kblk = gather_blocks((int)n);
    if (hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(h, DEM_E_HIP, "stream creation failed"));
    bool ok = hipMalloc(&h->tab64, sizeof(ShapeTab<double>) * p.n_shapes) == hipSuccess &&
              hipMalloc(&h->tab32, sizeof(ShapeTab<float>) * p.n_shapes) == hipSuccess &&
              hipMalloc(&h->ke_part, sizeof(double) * 2 * kblk) == hipSuccess &&
              hipMalloc(&h->e_part, sizeof(double) * 12 * h->nblk) == hipSuccess &&
              hipMalloc(&h->thermo, sizeof(double) * TH_COUNT) == hipSuccess &&
              hipMalloc(&h->stats, sizeof(unsigned long long) * ST_COUNT) == hipSuccess &&
              hipMalloc(&h->lst.flags, sizeof(int32_t) * FLAG_COUNT) == hipSuccess &&
              hipMalloc(&h->lst.cell_count, sizeof(int32_t) * sp.ncell) == hipSuccess &&
              hipMalloc(&h->lst.cell_start, sizeof(int32_t) * (sp.ncell + 1)) == hipSuccess &&
              hipMalloc(&h->lst.cell_particles, sizeof(int32_t) * n) == hipSuccess &&
              hipMalloc(&h->lst.pcell, sizeof(int32_t) * n) == hipSuccess &&
              hipMalloc(&h->lst.n_nbr, sizeof(int32_t) * n) == hipSuccess &&
              hipMalloc(&h->lst.xlast, sizeof(double) * 3 * n) == hipSuccess &&
              hipMalloc(&h->lst.klo, sizeof(int32_t) * n) == hipSuccess &&
              hipMalloc(&h->lst.pstart, sizeof(int32_t) * (n + 1)) == hipSuccess &&
              hipMalloc(&h->rot, (p.precision == DEM_FP32 ? sizeof(PartRec<float>) : sizeof(PartRec<double>)) * n) ==
                  hipSuccess;
    if (!ok) return bail(fail(h, DEM_E_OOM, "device allocation failed"));
    if (sp.n > 0) {  // shape ids index the LDS tables: validate before any kernel reads them
        std::vector<int32_t> sid((size_t)sp.n);
        if (hipMemcpyAsync(sid.data(), state->shape_id, sizeof(int32_t) * sid.size(), hipMemcpyDeviceToHost,
                           h->stream) != hipSuccess ||
            hipStreamSynchronize(h->stream) != hipSuccess)
            return bail(fail(h, DEM_E_HIP, "reading shape_id failed"));
        for (size_t i = 0; i < sid.size(); ++i)
            if (sid[i] < 0 || sid[i] >= p.n_shapes)
                return bail(fail(h, DEM_E_ARG, "shape_id[%zu] = %d outside [0, %d)", i, sid[i], p.n_shapes));
    }
    h->auto_cap = p.nbr_capacity <= 0;
    dem_status st = alloc_nbr(h, h->auto_cap ? auto_capacity(p, rl) : p.nbr_capacity);
    if (st != DEM_OK) return bail(st);
    // initial contents (not captured: plain memsets are fine here)
    if (hipMemcpyAsync(h->tab64, t64.data(), sizeof(ShapeTab<double>) * p.n_shapes, hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipMemcpyAsync(h->tab32, t32.data(), sizeof(ShapeTab<float>) * p.n_shapes, hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipMemsetAsync(h->lst.flags, 0, sizeof(int32_t) * FLAG_COUNT, h->stream) != hipSuccess ||
        hipMemsetAsync(h->lst.cell_count, 0, sizeof(int32_t) * sp.ncell, h->stream) != hipSuccess ||
        hipMemsetAsync(h->lst.n_nbr, 0, sizeof(int32_t) * n, h->stream) != hipSuccess ||
        hipMemsetAsync(h->stats, 0, sizeof(unsigned long long) * ST_COUNT, h->stream) != hipSuccess ||
        hipMemsetAsync(h->ke_part, 0, sizeof(double) * 2 * kblk, h->stream) != hipSuccess)
        return bail(fail(h, DEM_E_HIP, "initial upload failed"));
    k_set_thermo<<<1, 1, 0, h->stream>>>(h->thermo, 0.0, 0.0);
    if ((st = build_lists_sync(h)) != DEM_OK) return bail(st);
    if ((st = dem_compute_forces(h)) != DEM_OK) return bail(st);
    if ((st = dem_sync(h)) != DEM_OK) return bail(st);
    *out = h;
    return DEM_OK;
}

dem_status dem_destroy_system(dem_handle h)
{
    if (!h) return DEM_E_ARG;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    drop_graph(h);
    free_lists(h);
    (void)hipFree(h->lst.flags);
    (void)hipFree(h->tab64);
    (void)hipFree(h->tab32);
    (void)hipFree(h->ke_part);
    (void)hipFree(h->e_part);
    (void)hipFree(h->thermo);
    (void)hipFree(h->stats);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    delete h;
    return DEM_OK;
}

dem_status dem_build_celllist(dem_handle h)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    dem_status st = build_lists_sync(h);
    if (st != DEM_OK) return st;
    k_end_build<<<1, 1, 0, h->stream>>>(h->lst.flags);
    HIPCHK(h, hipGetLastError());
    return DEM_OK;
}

dem_status dem_compute_forces(dem_handle h)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    const ForcePtrs f = force_ptrs(h);
    launch_rotations(h->sp, h->st, h->rot, h->prm.precision, h->stream);
    launch_build_lists(h->sp, h->st, h->lst, h->stream);  // gated: only if a rebuild is due
    launch_pairs(h->sp, h->st, h->lst, f, h->prm.precision, h->stats, h->stream);
    launch_gather(h->sp, h->st, h->out, h->lst, f, h->prm.precision, false, h->ke_part, h->thermo, h->stream);
    HIPCHK(h, hipGetLastError());
    return DEM_OK;
}

dem_status dem_step(dem_handle h, int64_t n_steps)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    if (n_steps < 0) return fail(h, DEM_E_ARG, "n_steps < 0");
    if (n_steps == 0 || h->sp.n == 0) {
        h->step += n_steps;
        return DEM_OK;
    }
    dem_status st = ensure_graph(h);
    if (st != DEM_OK) return st;
    const bool nvt = h->sp.ensemble == DEM_NVT;
    if (nvt) {  // opening half step of the first step, from the current kinetic energy
        launch_kinetic(h->sp, h->st, h->ke_part, h->stream);
        launch_nh_begin(h->sp, h->ke_part, gather_blocks(h->sp.n), h->thermo, h->stream);
    }
    for (int64_t k = 0; k < n_steps; ++k) HIPCHK(h, hipGraphLaunch(h->gexec, h->stream));
    if (nvt) launch_nh_end(h->sp, h->st, h->ke_part, h->nblk, h->thermo, h->stream);
    HIPCHK(h, hipGetLastError());
    h->step += n_steps;
    return DEM_OK;
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
    std::memset(o, 0, sizeof *o);
    std::vector<double> part((size_t)12 * h->nblk, 0.0);
    double th[TH_COUNT];
    int32_t flags[FLAG_COUNT];
    launch_energy_partials(h->sp, h->st, h->out, h->e_part, h->stream);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipMemcpyAsync(part.data(), h->e_part, sizeof(double) * part.size(), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(th, h->thermo, sizeof th, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(flags, h->lst.flags, sizeof flags, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    double acc[12] = {0};
    if (h->sp.n > 0)
        for (int b = 0; b < h->nblk; ++b)
            for (int c = 0; c < 12; ++c) acc[c] += part[(size_t)12 * b + c];
    o->U = acc[0];
    o->K_trans = acc[1];
    o->K_rot = acc[2];
    for (int c = 0; c < 9; ++c) o->W[c] = acc[3 + c];
    const double K = o->K_trans + o->K_rot;
    o->T = h->sp.g > 0 ? 2.0 * K / h->sp.g : 0.0;
    const int d = h->sp.dim;
    const double vol = d == 3 ? h->sp.box[0] * h->sp.box[1] * h->sp.box[2] : h->sp.box[0] * h->sp.box[1];
    const double trW = d == 3 ? o->W[0] + o->W[4] + o->W[8] : o->W[0] + o->W[4];
    o->P = (2.0 * o->K_trans + trW) / (d * vol);
    o->xi = th[TH_XI];
    o->eta = th[TH_ETA];
    o->H = K + o->U;
    if (h->sp.ensemble == DEM_NVT) o->H += 0.5 * h->sp.Qm * o->xi * o->xi + h->sp.g * h->sp.kT * o->eta;
    o->step = h->step;
    o->n_rebuilds = flags[FLAG_NBUILDS];
    if (flags[FLAG_NONFINITE]) return fail(h, DEM_E_NONFINITE, "non-finite position or velocity");
    if (flags[FLAG_MAXROW] > h->sp.cap)
        return fail(h, DEM_E_CAPACITY, "neighbour row of %d exceeds capacity %d", flags[FLAG_MAXROW], h->sp.cap);
    return DEM_OK;
}

dem_status dem_set_thermostat(dem_handle h, double xi, double eta)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    k_set_thermo<<<1, 1, 0, h->stream>>>(h->thermo, xi, eta);
    HIPCHK(h, hipGetLastError());
    return DEM_OK;
}

dem_status dem_copy_lists(dem_handle h, int32_t *cell_start, int32_t *cell_particles, int32_t *nbr, int32_t *n_nbr,
                          int32_t *dims)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    const size_t n = (size_t)h->sp.n;
    if (cell_start)
        HIPCHK(h, hipMemcpyAsync(cell_start, h->lst.cell_start, sizeof(int32_t) * (h->sp.ncell + 1),
                                 hipMemcpyDeviceToHost, h->stream));
    if (cell_particles && n)
        HIPCHK(h, hipMemcpyAsync(cell_particles, h->lst.cell_particles, sizeof(int32_t) * n, hipMemcpyDeviceToHost,
                                 h->stream));
    if (nbr && n)
        HIPCHK(h, hipMemcpyAsync(nbr, h->lst.nbr, sizeof(int32_t) * n * h->sp.cap, hipMemcpyDeviceToHost, h->stream));
    if (n_nbr && n)
        HIPCHK(h, hipMemcpyAsync(n_nbr, h->lst.n_nbr, sizeof(int32_t) * n, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (dims) {
        dims[0] = h->sp.nc[0];
        dims[1] = h->sp.nc[1];
        dims[2] = h->sp.nc[2];
        dims[3] = h->sp.cap;
    }
    return DEM_OK;
}

dem_status dem_list_info(dem_handle h, double *r_list, int32_t *n_cells, int32_t *capacity)
{
    if (!h) return fail(nullptr, DEM_E_ARG, "null handle");
    if (r_list) *r_list = h->r_list;
    if (n_cells) *n_cells = h->sp.ncell;
    if (capacity) *capacity = h->sp.cap;
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
    hipEvent_t e0, e1;
    HIPCHK(h, hipEventCreate(&e0));
    HIPCHK(h, hipEventCreate(&e1));
    const ForcePtrs f = force_ptrs(h);
    launch_pairs(h->sp, h->st, h->lst, f, h->prm.precision, nullptr, h->stream);  // warm
    HIPCHK(h, hipEventRecord(e0, h->stream));
    for (int r = 0; r < reps; ++r) launch_pairs(h->sp, h->st, h->lst, f, h->prm.precision, nullptr, h->stream);
    HIPCHK(h, hipEventRecord(e1, h->stream));
    HIPCHK(h, hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHK(h, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *mean_ms = (double)ms / reps;
    return DEM_OK;
}

}  // extern "C"

// Cell list, full neighbour list and half pair list of every replica.
//
// The lists are an integer contract: the cell of a particle is
// min(n_c - 1, floor(x / (L / n_c))) per axis, cells are CSR with particles
// ascending inside a cell, and the neighbours of i are every j != i of the
// same replica with |minimum image (x_j - x_i)|^2 < r_list^2, evaluated in
// FP64 as written (no contraction into fused multiply-adds), stored
// ascending in j.  Rows live column-major (nbr[k * N + i]) so per-row loads
// are contiguous across particles.  The half list enumerates each unordered
// pair once (owner i < j) with the row slot it occupies in both rows, so
// the force pass evaluates a pair once, writes its result into both slots,
// and each particle sums its own row.
//
// Every list kernel returns at once unless a rebuild is pending, so a
// captured step contains the build unconditionally.  Replicas of up to
// kFusedMaxN particles build everything in one workgroup each (one launch
// per step for the whole batch, the phases separated by workgroup
// barriers); a single larger system uses one grid-wide kernel per phase.
// Both run the same per-item code.  After a build the pair kernel's tile
// plan (the first tile of each replica) is recomputed.
#include "dem_internal.h"

#pragma clang fp contract(off)

namespace dem {
namespace {

constexpr int kFusedMaxN = 65536;

__device__ inline int cell_coord(double x, double w, int nc)
{
    int c = (int)floor(x / w);
    c = c < 0 ? 0 : c;
    return c > nc - 1 ? nc - 1 : c;
}

// Minimum image of d = x_j - x_i for positions in [0, L].  This equals
// d - L rint(d / L) bit for bit except where |d| is within rounding of L/2,
// and there both forms give |d| >= L/2 >= r_list, so no list decision can
// differ; it avoids an FP64 division per candidate.
__device__ inline double min_image(double d, double L)
{
    const double h = 0.5 * L;
    return d > h ? d - L : (d < -h ? d + L : d);
}

// ---- per-item steps (i, j: global particle slots; cells: replica-local) ----
__device__ inline void cell_assign(const SysParams &p, const StatePtrs &s, const ListPtrs &l, int i)
{
    const int cx = cell_coord(s.x[i], p.cellw[0], p.nc[0]);
    const int cy = cell_coord(s.y[i], p.cellw[1], p.nc[1]);
    const int cz = (p.dim == 3) ? cell_coord(s.z[i], p.cellw[2], p.nc[2]) : 0;
    const int c = cx + p.nc[0] * (cy + p.nc[1] * cz);
    l.pcell[i] = c;
    atomicAdd(&l.cell_count[p.coff + c], 1);
}

// Scatter; counting each cell back down leaves cell_count zeroed for the next build.
__device__ inline void cell_fill(const SysParams &p, const ListPtrs &l, int i)
{
    const int c = l.pcell[i];
    const int slot = atomicSub(&l.cell_count[p.coff + c], 1) - 1;
    l.cell_particles[p.off + l.cell_start[p.coff + c] + slot] = i;
}

// The scatter order is arbitrary: sort every cell ascending (cells hold a few particles).
__device__ inline void cell_sort(const SysParams &p, const ListPtrs &l, int c)
{
    const int lo = p.off + l.cell_start[p.coff + c], hi = p.off + l.cell_start[p.coff + c + 1];
    for (int a = lo + 1; a < hi; ++a) {
        const int key = l.cell_particles[a];
        int b = a - 1;
        while (b >= lo && l.cell_particles[b] > key) {
            l.cell_particles[b + 1] = l.cell_particles[b];
            --b;
        }
        l.cell_particles[b + 1] = key;
    }
}

__device__ inline bool within(const SysParams &p, const StatePtrs &s, double xi, double yi, double zi, int j)
{
    const double dx = min_image(s.x[j] - xi, p.box[0]);
    const double dy = min_image(s.y[j] - yi, p.box[1]);
    double r2 = dx * dx + dy * dy;
    if (p.dim == 3) {
        const double dz = min_image(s.z[j] - zi, p.box[2]);
        r2 = r2 + dz * dz;
    }
    return r2 < p.rl2;
}

__device__ inline void nbr_build(const SysParams &p, const BatchParams &b, const StatePtrs &s, const ListPtrs &l, int i)
{
    const size_t N = (size_t)b.N;
    const int cap = b.cap;
    const double xi = s.x[i], yi = s.y[i], zi = (p.dim == 3) ? s.z[i] : 0.0;
    int count = 0;
    if (p.use_cells) {
        const int c = l.pcell[i];
        const int cx = c % p.nc[0];
        const int cy = (c / p.nc[0]) % p.nc[1];
        const int cz = c / (p.nc[0] * p.nc[1]);
        const int zlo = (p.dim == 3) ? -1 : 0, zhi = (p.dim == 3) ? 1 : 0;
        for (int dz = zlo; dz <= zhi; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int ax = cx + dx, ay = cy + dy, az = cz + dz;
                    ax += (ax < 0) ? p.nc[0] : 0;
                    ax -= (ax >= p.nc[0]) ? p.nc[0] : 0;
                    ay += (ay < 0) ? p.nc[1] : 0;
                    ay -= (ay >= p.nc[1]) ? p.nc[1] : 0;
                    az += (az < 0) ? p.nc[2] : 0;
                    az -= (az >= p.nc[2]) ? p.nc[2] : 0;
                    const int cc = p.coff + ax + p.nc[0] * (ay + p.nc[1] * az);
                    for (int t = p.off + l.cell_start[cc]; t < p.off + l.cell_start[cc + 1]; ++t) {
                        const int j = l.cell_particles[t];
                        if (j != i && within(p, s, xi, yi, zi, j)) {
                            if (count < cap) l.nbr[(size_t)count * N + i] = j;
                            ++count;
                        }
                    }
                }
    } else {
        for (int j = p.off; j < p.off + p.n; ++j)
            if (j != i && within(p, s, xi, yi, zi, j)) {
                if (count < cap) l.nbr[(size_t)count * N + i] = j;
                ++count;
            }
    }
    const int m = count < cap ? count : cap;
    for (int a = 1; a < m; ++a) {  // ascending row
        const int key = l.nbr[(size_t)a * N + i];
        int c = a - 1;
        while (c >= 0 && l.nbr[(size_t)c * N + i] > key) {
            l.nbr[(size_t)(c + 1) * N + i] = l.nbr[(size_t)c * N + i];
            --c;
        }
        l.nbr[(size_t)(c + 1) * N + i] = key;
    }
    l.n_nbr[i] = m;
    if (count > cap) atomicMax(&l.flags[p.rid * FLAG_COUNT + FLAG_MAXROW], count);
    l.xlast[i] = xi;
    l.xlast[N + i] = yi;
    l.xlast[2 * N + i] = zi;
}

// First slot of row i holding a neighbour j > i (rows ascend), and the
// number of such slots: i owns the pairs (i, j > i) of the half list.
__device__ inline void pair_count(const BatchParams &b, const ListPtrs &l, int32_t *upper, int i)
{
    const size_t N = (size_t)b.N;
    const int m = l.n_nbr[i];
    int lo = 0, hi = m;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (l.nbr[(size_t)mid * N + i] > i) hi = mid;
        else lo = mid + 1;
    }
    l.klo[i] = lo;
    upper[i] = m - lo;
}

// Pair entries: the owner i of pair q writes {i, j, slot of j in i's row,
// slot of i in j's row} with one store, the last found by bisection in j's
// row (-1 if a row overflow left i out of it, which is reported).  Pair
// indices are local to the replica.
__device__ inline void pair_fill(const SysParams &p, const BatchParams &b, const ListPtrs &l, int i)
{
    const size_t N = (size_t)b.N;
    const int m = l.n_nbr[i], k0 = l.klo[i];
    int4 *pairs = l.pairs + p.poff;
    for (int k = k0; k < m; ++k) {
        const int q = l.pstart[i] + (k - k0);
        if (q >= p.pcap) break;  // (only after a row overflow, which is reported)
        const int j = l.nbr[(size_t)k * N + i];
        int lo = 0, hi = l.klo[j];  // j's neighbours below j, ascending
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (l.nbr[(size_t)mid * N + j] < i) lo = mid + 1;
            else hi = mid;
        }
        const int w = (lo < l.klo[j] && l.nbr[(size_t)lo * N + j] == i) ? lo : -1;
        pairs[q] = make_int4(i, j, k, w);
    }
}

// Exclusive scan of count[0..m) into start[0..m) by one workgroup of 1024
// threads; returns the total to every thread.  count and start may alias.
__device__ inline int block_scan(const int32_t *count, int32_t *start, int m, int *part)
{
    const int t = threadIdx.x;
    const int per = (m + 1023) / 1024;
    const int lo = t * per, hi = min(lo + per, m);
    int sum = 0;
    for (int c = lo; c < hi; ++c) sum += count[c];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = (t >= off) ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - sum;
    for (int c = lo; c < hi; ++c) {
        const int cnt = count[c];
        start[c] = run;
        run += cnt;
    }
    const int total = part[1023];
    __syncthreads();
    return total;
}

// ---- one kernel per phase (a single replica, slot 0) -----------------------
__global__ void k_cell_assign(SysParams p, StatePtrs s, ListPtrs l)
{
    if (l.flags[FLAG_REBUILD] == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p.n) cell_assign(p, s, l, i);
}

__global__ void __launch_bounds__(1024) k_scan(const int32_t *count, int32_t *start, int m, const int32_t *flags)
{
    if (flags[FLAG_REBUILD] == 0) return;
    __shared__ int part[1024];
    const int total = block_scan(count, start, m, part);
    if (threadIdx.x == 0) start[m] = total;
}

__global__ void k_cell_fill(SysParams p, ListPtrs l)
{
    if (l.flags[FLAG_REBUILD] == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p.n) cell_fill(p, l, i);
}

__global__ void k_cell_sort(SysParams p, ListPtrs l)
{
    if (l.flags[FLAG_REBUILD] == 0) return;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < p.ncell) cell_sort(p, l, c);
}

__global__ void k_nbr_build(SysParams p, BatchParams b, StatePtrs s, ListPtrs l)
{
    if (l.flags[FLAG_REBUILD] == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p.n) nbr_build(p, b, s, l, i);
}

__global__ void k_pair_count(SysParams p, BatchParams b, ListPtrs l)
{
    if (l.flags[FLAG_REBUILD] == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p.n) pair_count(b, l, l.pcell, i);  // pcell is free after the neighbour build
}

__global__ void k_pair_fill(SysParams p, BatchParams b, ListPtrs l)
{
    if (l.flags[FLAG_REBUILD] == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        const int np = min(l.pstart[p.n], p.pcap);
        l.flags[FLAG_NPAIRS] = np;
        l.tile_start[0] = 0;
        l.tile_start[1] = (np + kTile - 1) / kTile;
        l.gflags[G_ANY] = 0;
    }
    if (i < p.n) pair_fill(p, b, l, i);
}

// ---- the whole build of one replica per workgroup ---------------------------
// Workgroup r rebuilds replica r if its flag is set; the last workgroup to
// finish recomputes the tile plan over all replicas.
__global__ void __launch_bounds__(1024) k_lists_fused(BatchParams b, const SysParams *reps, StatePtrs s, ListPtrs l)
{
    if (l.gflags[G_ANY] == 0) return;
    __shared__ int part[1024];
    __shared__ int last;
    const int t = threadIdx.x;
    const SysParams &p = reps[blockIdx.x];
    int32_t *fl = l.flags + blockIdx.x * FLAG_COUNT;
    if (p.live && p.n > 0 && fl[FLAG_REBUILD] != 0) {
        const int lo = p.off, hi = p.off + p.n;
        for (int i = lo + t; i < hi; i += 1024) cell_assign(p, s, l, i);
        __syncthreads();
        const int ncp = block_scan(l.cell_count + p.coff, l.cell_start + p.coff, p.ncell, part);
        if (t == 0) l.cell_start[p.coff + p.ncell] = ncp;
        for (int i = lo + t; i < hi; i += 1024) cell_fill(p, l, i);
        __syncthreads();
        for (int c = t; c < p.ncell; c += 1024) cell_sort(p, l, c);
        __syncthreads();
        for (int i = lo + t; i < hi; i += 1024) nbr_build(p, b, s, l, i);
        __syncthreads();
        for (int i = lo + t; i < hi; i += 1024) pair_count(b, l, l.pcell, i);
        __syncthreads();
        const int np = block_scan(l.pcell + p.off, l.pstart + p.off, p.n, part);
        for (int i = lo + t; i < hi; i += 1024) pair_fill(p, b, l, i);
        if (t == 0) fl[FLAG_NPAIRS] = min(np, p.pcap);
    }
    __syncthreads();
    if (t == 0) {
        __threadfence();
        last = atomicAdd(&l.gflags[G_TICKET], 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    // tiles per replica, then their exclusive scan in place
    const volatile int32_t *vfl = l.flags;
    for (int r = t; r < b.nrep; r += 1024) {
        const int np = vfl[r * FLAG_COUNT + FLAG_NPAIRS];
        l.tile_start[r] = reps[r].live ? (np + kTile - 1) / kTile : 0;
    }
    __syncthreads();
    const int total = block_scan(l.tile_start, l.tile_start, b.nrep, part);
    if (t == 0) {
        l.tile_start[b.nrep] = total;
        l.gflags[G_ANY] = 0;
        l.gflags[G_TICKET] = 0;
    }
}

}  // namespace

void launch_build_lists(const Launch &L, int multi, const SysParams &p, hipStream_t stream)
{
    if (L.b.nrep == 0) return;
    if (!multi) {
        k_lists_fused<<<L.b.nrep, 1024, 0, stream>>>(L.b, L.reps, L.s, L.l);
        return;
    }
    if (p.n == 0) return;
    const int nb = blocks_for(p.n);
    k_cell_assign<<<nb, kBlock, 0, stream>>>(p, L.s, L.l);
    k_scan<<<1, 1024, 0, stream>>>(L.l.cell_count, L.l.cell_start, p.ncell, L.l.flags);
    k_cell_fill<<<nb, kBlock, 0, stream>>>(p, L.l);
    k_cell_sort<<<blocks_for(p.ncell), kBlock, 0, stream>>>(p, L.l);
    k_nbr_build<<<nb, kBlock, 0, stream>>>(p, L.b, L.s, L.l);
    k_pair_count<<<nb, kBlock, 0, stream>>>(p, L.b, L.l);
    k_scan<<<1, 1024, 0, stream>>>(L.l.pcell, L.l.pstart, p.n, L.l.flags);
    k_pair_fill<<<nb, kBlock, 0, stream>>>(p, L.b, L.l);
}

int fused_list_max_n() { return kFusedMaxN; }

}  // namespace dem

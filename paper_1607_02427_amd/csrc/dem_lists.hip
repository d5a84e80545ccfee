// Cell list, full neighbour list and half pair list.
//
// The lists are an integer contract: the cell of a particle is
// min(n_c - 1, floor(x / (L / n_c))) per axis, cells are CSR with particles
// ascending inside a cell, and the neighbours of i are every j != i with
// |minimum image (x_j - x_i)|^2 < r_list^2, evaluated in FP64 as written
// (no contraction into fused multiply-adds), stored ascending in j.
// Rows live column-major (nbr[k * n + i]) so per-row loads are contiguous
// across particles.  The half list enumerates each unordered pair once
// (owner i < j) with the row slot it occupies in both rows, so the force
// pass evaluates a pair once, writes its result into both slots, and each
// particle sums its own row.
//
// Every list kernel returns at once unless the rebuild flag is set, so a
// captured step contains the build unconditionally.  Systems of up to
// kFusedMaxN particles build everything in one workgroup (one launch per
// step, the phases separated by workgroup barriers); larger systems use one
// grid-wide kernel per phase.  Both run the same per-item code.
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

// ---- per-item steps --------------------------------------------------------
__device__ inline void cell_assign(const SysParams &p, const StatePtrs &s, const ListPtrs &l, int i)
{
    const int cx = cell_coord(s.x[i], p.cellw[0], p.nc[0]);
    const int cy = cell_coord(s.y[i], p.cellw[1], p.nc[1]);
    const int cz = (p.dim == 3) ? cell_coord(s.z[i], p.cellw[2], p.nc[2]) : 0;
    const int c = cx + p.nc[0] * (cy + p.nc[1] * cz);
    l.pcell[i] = c;
    atomicAdd(&l.cell_count[c], 1);
}

// Scatter; counting each cell back down leaves cell_count zeroed for the next build.
__device__ inline void cell_fill(const ListPtrs &l, int i)
{
    const int c = l.pcell[i];
    const int slot = atomicSub(&l.cell_count[c], 1) - 1;
    l.cell_particles[l.cell_start[c] + slot] = i;
}

// The scatter order is arbitrary: sort every cell ascending (cells hold a few particles).
__device__ inline void cell_sort(const ListPtrs &l, int c)
{
    const int lo = l.cell_start[c], hi = l.cell_start[c + 1];
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

__device__ inline void nbr_build(const SysParams &p, const StatePtrs &s, const ListPtrs &l, int i)
{
    const int n = p.n;
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
                    const int cc = ax + p.nc[0] * (ay + p.nc[1] * az);
                    for (int t = l.cell_start[cc]; t < l.cell_start[cc + 1]; ++t) {
                        const int j = l.cell_particles[t];
                        if (j != i && within(p, s, xi, yi, zi, j)) {
                            if (count < p.cap) l.nbr[(size_t)count * n + i] = j;
                            ++count;
                        }
                    }
                }
    } else {
        for (int j = 0; j < n; ++j)
            if (j != i && within(p, s, xi, yi, zi, j)) {
                if (count < p.cap) l.nbr[(size_t)count * n + i] = j;
                ++count;
            }
    }
    const int m = count < p.cap ? count : p.cap;
    for (int a = 1; a < m; ++a) {  // ascending row
        const int key = l.nbr[(size_t)a * n + i];
        int b = a - 1;
        while (b >= 0 && l.nbr[(size_t)b * n + i] > key) {
            l.nbr[(size_t)(b + 1) * n + i] = l.nbr[(size_t)b * n + i];
            --b;
        }
        l.nbr[(size_t)(b + 1) * n + i] = key;
    }
    l.n_nbr[i] = m;
    if (count > p.cap) atomicMax(&l.flags[FLAG_MAXROW], count);
    l.xlast[i] = xi;
    l.xlast[n + i] = yi;
    l.xlast[2 * n + i] = zi;
}

// First slot of row i holding a neighbour j > i (rows ascend), and the
// number of such slots: i owns the pairs (i, j > i) of the half list.
__device__ inline void pair_count(const SysParams &p, const ListPtrs &l, int32_t *upper, int i)
{
    const int n = p.n, m = l.n_nbr[i];
    int lo = 0, hi = m;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (l.nbr[(size_t)mid * n + i] > i) hi = mid;
        else lo = mid + 1;
    }
    l.klo[i] = lo;
    upper[i] = m - lo;
}

// Pair arrays and, for every pair, the row slot it occupies in each of the
// two rows; a slot (k, i) with j < i belongs to the pair owned by j, found
// by bisection in j's row.
__device__ inline void pair_fill(const SysParams &p, const ListPtrs &l, int i)
{
    const int n = p.n, m = l.n_nbr[i], k0 = l.klo[i];
    for (int k = 0; k < m; ++k) {
        const int j = l.nbr[(size_t)k * n + i];
        int q = -1;
        if (k >= k0) {
            q = l.pstart[i] + (k - k0);
            if (q < p.max_pairs) {  // (q beyond the capacity only after a row overflow, which is reported)
                l.pairs[q].x = i;
                l.pairs[q].y = j;
                l.pairs[q].z = k;
            }
        } else {
            int lo = l.klo[j], hi = l.n_nbr[j];
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (l.nbr[(size_t)mid * n + j] < i) lo = mid + 1;
                else hi = mid;
            }
            if (lo < l.n_nbr[j] && l.nbr[(size_t)lo * n + j] == i) q = l.pstart[j] + (lo - l.klo[j]);
            if (q >= 0 && q < p.max_pairs) l.pairs[q].w = k;
        }
    }
}

// Exclusive scan of count[0..m) into start[0..m], start[m] = total, by one
// workgroup of 1024 threads.
__device__ inline void block_scan(const int32_t *count, int32_t *start, int m, int *part)
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
        start[c] = run;
        run += count[c];
    }
    if (t == 1023) start[m] = part[1023];
    __syncthreads();
}

// ---- grid-wide kernels (one per phase) -------------------------------------
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
    block_scan(count, start, m, part);
}

__global__ void k_cell_fill(SysParams p, ListPtrs l)
{
    if (l.flags[FLAG_REBUILD] == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p.n) cell_fill(l, i);
}

__global__ void k_cell_sort(SysParams p, ListPtrs l)
{
    if (l.flags[FLAG_REBUILD] == 0) return;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < p.ncell) cell_sort(l, c);
}

__global__ void k_nbr_build(SysParams p, StatePtrs s, ListPtrs l)
{
    if (l.flags[FLAG_REBUILD] == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p.n) nbr_build(p, s, l, i);
}

__global__ void k_pair_count(SysParams p, ListPtrs l)
{
    if (l.flags[FLAG_REBUILD] == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p.n) pair_count(p, l, l.pcell, i);  // pcell is free after the neighbour build
}

__global__ void k_pair_fill(SysParams p, ListPtrs l)
{
    if (l.flags[FLAG_REBUILD] == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) l.flags[FLAG_NPAIRS] = min(l.pstart[p.n], p.max_pairs);
    if (i < p.n) pair_fill(p, l, i);
}

// ---- the whole build in one workgroup ---------------------------------------
__global__ void __launch_bounds__(1024) k_lists_fused(SysParams p, StatePtrs s, ListPtrs l)
{
    if (l.flags[FLAG_REBUILD] == 0) return;
    __shared__ int part[1024];
    const int t = threadIdx.x, n = p.n;
    for (int i = t; i < n; i += 1024) cell_assign(p, s, l, i);
    __syncthreads();
    block_scan(l.cell_count, l.cell_start, p.ncell, part);
    for (int i = t; i < n; i += 1024) cell_fill(l, i);
    __syncthreads();
    for (int c = t; c < p.ncell; c += 1024) cell_sort(l, c);
    __syncthreads();
    for (int i = t; i < n; i += 1024) nbr_build(p, s, l, i);
    __syncthreads();
    for (int i = t; i < n; i += 1024) pair_count(p, l, l.pcell, i);
    __syncthreads();
    block_scan(l.pcell, l.pstart, n, part);
    if (t == 0) l.flags[FLAG_NPAIRS] = min(l.pstart[n], p.max_pairs);
    for (int i = t; i < n; i += 1024) pair_fill(p, l, i);
}

}  // namespace

void launch_build_lists(const SysParams &p, const StatePtrs &s, const ListPtrs &l, hipStream_t stream)
{
    if (p.n == 0) return;
    if (p.n <= kFusedMaxN && !p.force_multi_kernel_lists) {
        k_lists_fused<<<1, 1024, 0, stream>>>(p, s, l);
        return;
    }
    const int nb = blocks_for(p.n);
    k_cell_assign<<<nb, kBlock, 0, stream>>>(p, s, l);
    k_scan<<<1, 1024, 0, stream>>>(l.cell_count, l.cell_start, p.ncell, l.flags);
    k_cell_fill<<<nb, kBlock, 0, stream>>>(p, l);
    k_cell_sort<<<blocks_for(p.ncell), kBlock, 0, stream>>>(p, l);
    k_nbr_build<<<nb, kBlock, 0, stream>>>(p, s, l);
    k_pair_count<<<nb, kBlock, 0, stream>>>(p, l);
    k_scan<<<1, 1024, 0, stream>>>(l.pcell, l.pstart, p.n, l.flags);
    k_pair_fill<<<nb, kBlock, 0, stream>>>(p, l);
}

}  // namespace dem

// Device parts of a list build, shared by the list kernels of a build
// outside a step (dem_lists.hip) and by the step kernels that carry a build
// inside a step (dem_force.hip):
//   * nbr_rows: the neighbour rows of 4 particles by one wavefront (16
//     lanes per particle);
//   * fill_chunk: the pair offsets and pair entries of one chunk by one
//     wavefront;
//   * plan: the tile plan of the pair kernel by one workgroup.
// The list decisions are an integer contract: |minimum image (x_j -
// x_i)|^2 < r_list^2 evaluated in FP64 as written, with no contraction into
// fused multiply-adds (the pragma at the top of each function body that
// evaluates them).
#pragma once

#include "dem_internal.h"

namespace dem {
namespace lb {

constexpr int kNbrLanes = 16;                 // lanes per particle in nbr_rows
constexpr int kNbrPer = lb_rows_per_group;    // particles per nbr_rows wavefront
static_assert(kNbrPer * kNbrLanes == 64, "one wavefront per group of particles");

// Minimum image of d = x_j - x_i for positions in [0, L].  This equals
// d - L rint(d / L) bit for bit except where |d| is within rounding of L/2,
// and there both forms give |d| >= L/2 >= r_list, so no list decision can
// differ; it avoids an FP64 division per candidate.
__device__ inline double min_image(double d, double L)
{
    const double h = 0.5 * L;
    return d > h ? d - L : (d < -h ? d + L : d);
}

__device__ inline bool within(const SysParams &p, const StatePtrs &s, double xi, double yi, double zi, int j)
{
#pragma clang fp contract(off)
    const double dx = min_image(s.x[j] - xi, p.box[0]);
    const double dy = min_image(s.y[j] - yi, p.box[1]);
    double r2 = dx * dx + dy * dy;
    if (p.dim == 3) {
        const double dz = min_image(s.z[j] - zi, p.box[2]);
        r2 = r2 + dz * dz;
    }
    return r2 < p.rl2;
}

__device__ inline unsigned long long lanes_below()
{
    const unsigned lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Does this build take replica r?  (LISTS_REFILL: every live replica that
// has lists; LISTS_STEP: a replica whose step rebuilds and has steps left.)
__device__ inline bool building(int mode, int r, const SysParams &p, const int32_t *fl, const int64_t *budget)
{
    if (!p.live) return false;
    if (mode == LISTS_STEP) return fl[FLAG_REBUILD] != 0 && budget[r] > 0;
    if (mode == LISTS_REFILL) return fl[FLAG_NBUILDS] > 0;
    return mode == LISTS_ALL || mode == r;
}

// Exclusive scan of count[0..m) into start[0..m) by one workgroup of NT
// threads (count may be start; it is read through volatile loads, as other
// workgroups wrote it); part holds NT ints of LDS.  Returns the total.
template <int NT>
__device__ int block_scan(const int32_t *count, int32_t *start, int m, int *part)
{
    const volatile int32_t *vc = count;
    const int t = threadIdx.x;
    const int per = (m + NT - 1) / NT;
    const int lo = min(t * per, m), hi = min(lo + per, m);
    int sum = 0;
    for (int c = lo; c < hi; ++c) sum += vc[c];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
        const int v = (t >= off) ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - sum;
    for (int c = lo; c < hi; ++c) {
        const int cnt = vc[c];
        start[c] = run;
        run += cnt;
    }
    const int total = part[NT - 1];
    __syncthreads();
    return total;
}

// Neighbour rows of particles 4 vb .. 4 vb + 3 (all of one chunk, so of one
// replica), by one wavefront (a workgroup of 64 threads; the caller has
// checked that the replica builds).  Each lane scans some of
// the neighbour cells (or, without cells, a sixteenth of the replica); hits
// are appended to the particle's LDS buffer in ballot order, then every
// kept hit finds its rank (the number of smaller hits) and is stored in
// that row slot, so the row ascends and keeps the cap smallest j.  The row's
// count of j > i is the particle's pair count; the wavefront stores its
// total as ptot[vb] and adds it to the replica's FLAG_NEWPAIRS (cleared when
// the build starts).  buf: kNbrPer * kRowMax ints of LDS.
template <int DIM>
__device__ void nbr_rows(const BatchParams &b, const SysParams &p, const StatePtrs &s, const ListPtrs &l, int32_t *fl,
                         int vb, int *buf)
{
    const int g = threadIdx.x / kNbrLanes, sub = threadIdx.x % kNbrLanes;
    const int i = vb * kNbrPer + g;
    int *row = buf + g * kRowMax;
    const bool mine = i < p.off + p.n;
    const unsigned long long gmask = 0xffffull << (kNbrLanes * ((threadIdx.x & 63) / kNbrLanes));
    const unsigned long long below = lanes_below();
    const double xi = mine ? s.x[i] : 0.0, yi = mine ? s.y[i] : 0.0, zi = (mine && DIM == 3) ? s.z[i] : 0.0;
    int m = 0;  // hits so far (the same in all lanes of the particle)
    if (p.use_cells) {
        const int c = mine ? l.pcell[i] : 0;
        const int cx = c % p.nc[0], cy = (c / p.nc[0]) % p.nc[1], cz = c / (p.nc[0] * p.nc[1]);
        constexpr int kNb = DIM == 3 ? 27 : 9;
        for (int t0 = 0; t0 < kNb; t0 += kNbrLanes) {
            const int t = t0 + sub;
            int cc = 0, cnt = 0;
            if (mine && t < kNb) {
                int ax = cx + t % 3 - 1, ay = cy + (t / 3) % 3 - 1, az = cz + (DIM == 3 ? t / 9 - 1 : 0);
                ax += (ax < 0) ? p.nc[0] : 0;
                ax -= (ax >= p.nc[0]) ? p.nc[0] : 0;
                ay += (ay < 0) ? p.nc[1] : 0;
                ay -= (ay >= p.nc[1]) ? p.nc[1] : 0;
                az += (az < 0) ? p.nc[2] : 0;
                az -= (az >= p.nc[2]) ? p.nc[2] : 0;
                cc = p.coff + ax + p.nc[0] * (ay + p.nc[1] * az);
                cnt = min(l.cell_count[cc], kCellCap);
            }
            for (int k = 0;; ++k) {
                const bool has = k < cnt;
                if (__ballot(has) == 0) break;
                int j = 0;
                bool hit = false;
                if (has) {
                    j = l.cell_slot[(size_t)cc * kCellCap + k];
                    hit = j != i && within(p, s, xi, yi, zi, j);
                }
                const unsigned long long hm = __ballot(hit);
                const int pos = m + __popcll(hm & below & gmask);
                if (hit && pos < kRowMax) row[pos] = j;
                m += __popcll(hm & gmask);
            }
        }
    } else {
        for (int k0 = 0; k0 < p.n; k0 += kNbrLanes) {
            const int j = p.off + k0 + sub;
            const bool hit = mine && k0 + sub < p.n && j != i && within(p, s, xi, yi, zi, j);
            const unsigned long long hm = __ballot(hit);
            const int pos = m + __popcll(hm & below & gmask);
            if (hit && pos < kRowMax) row[pos] = j;
            m += __popcll(hm & gmask);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const size_t N = (size_t)b.N;
    const int cap = b.cap;
    const int mm = min(m, kRowMax);
    int lower = 0;  // kept hits below i
    if (mine)
        for (int e = sub; e < mm; e += kNbrLanes) {
            const int v = row[e];
            int rank = 0;
            for (int f = 0; f < mm; ++f) rank += row[f] < v ? 1 : 0;
            if (rank < cap) {
                l.nbr[(size_t)rank * N + i] = v;
                lower += v < i ? 1 : 0;
            }
        }
    for (int off = kNbrLanes / 2; off > 0; off >>= 1) lower += __shfl_xor(lower, off, kNbrLanes);
    const int kept = min(m, cap);
    if (mine && sub == 0) {
        l.n_nbr[i] = kept;
        l.klo[i] = lower;
        l.pstart[i] = kept - lower;  // pair count; fill_chunk turns it into an offset
        if (m > cap) atomicMax(&fl[FLAG_MAXROW], m);
        l.xlast[i] = xi;
        l.xlast[N + i] = yi;
        l.xlast[2 * N + i] = zi;
    }
    // the wavefront's pair count, for the pair offsets and (an integer sum,
    // in any order) the replica's total
    int tot = (mine && sub == 0) ? kept - lower : 0;
    for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off, 64);
    if (threadIdx.x == 0) {
        l.ptot[vb] = tot;
        atomicAdd(&fl[FLAG_NEWPAIRS], tot);
    }
    // buf is free for the next call once every lane has read it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pair entries: the owner i of pair q writes {i, j, slot of j in i's row,
// slot of i in j's row} with one store, the last found by bisection in j's
// row (-1 if a row overflow left i out of it, which is reported).
__device__ inline void pair_fill(const SysParams &p, const BatchParams &b, const ListPtrs &l, int i)
{
    const size_t N = (size_t)b.N;
    const int m = min(l.n_nbr[i], b.cap), k0 = max(l.klo[i], 0);
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

// Pair offsets (unless `refill`: the offsets are kept) and pair entries of
// chunk c of replica p, by one wavefront (lane = particle c * 64 + lane),
// then the chunk's cells emptied when `clear_cells`.  The offset of i is the
// counts of the replica's row groups (ptot) before this chunk plus the
// counts of the chunk's particles before i.
__device__ inline void fill_chunk(const BatchParams &b, const SysParams &p, const ListPtrs &l, int c, bool refill,
                                  bool clear_cells)
{
    const int lane = __lane_id();
    const int i = c * kChunk + lane;
    const bool mine = i < p.off + p.n;
    if (!refill) {
        const int cnt = mine ? l.pstart[i] : 0;
        int incl = cnt;
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off, 64);
            if (lane >= off) incl += v;
        }
        int prior = 0;
#pragma unroll 8
        for (int q = p.off / kNbrPer + lane; q < c * (kChunk / kNbrPer); q += 64) prior += l.ptot[q];
        for (int off = 32; off > 0; off >>= 1) prior += __shfl_xor(prior, off, 64);
        if (mine) l.pstart[i] = prior + incl - cnt;
    }
    if (!mine) return;
    pair_fill(p, b, l, i);
    // every particle of the cell writes the same zero (without cells the
    // word is zero already; use_cells of a replica under the barostat may
    // change while this runs)
    if (clear_cells) l.cell_count[p.coff + l.pcell[i]] = 0;
}

// Tile plan (the first tile of each replica, b.tile pairs per tile) by one
// workgroup of NT threads; a replica for which built(r) holds takes its new
// pair total (FLAG_NEWPAIRS) first.  part: NT ints of LDS.
template <int NT, typename Built>
__device__ void plan(const BatchParams &b, const SysParams *reps, const ListPtrs &l, int *part, Built built)
{
    const volatile int32_t *vfl = l.flags;
    for (int r = threadIdx.x; r < b.nrep; r += NT) {
        int np = vfl[r * FLAG_COUNT + FLAG_NPAIRS];
        if (reps[r].live && built(r)) np = vfl[r * FLAG_COUNT + FLAG_NEWPAIRS];
        np = min(np, reps[r].pcap);  // (above pcap only after an overflow)
        l.flags[r * FLAG_COUNT + FLAG_NPAIRS] = np;
        l.tile_start[r] = reps[r].live ? (np + b.tile - 1) / b.tile : 0;
    }
    __syncthreads();
    const int total = block_scan<NT>(l.tile_start, l.tile_start, b.nrep, part);
    if (threadIdx.x == 0) l.tile_start[b.nrep] = total;
}

}  // namespace lb
}  // namespace dem

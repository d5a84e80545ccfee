// Cell list, full neighbour list and half pair list of every replica, built
// across the whole device.
//
// The lists are an integer contract: the cell of a particle is
// min(n_c - 1, floor(x / (L / n_c))) per axis, and the neighbours of i are
// every j != i of the same replica with |minimum image (x_j - x_i)|^2 <
// r_list^2, evaluated in FP64 as written (no contraction into fused
// multiply-adds), stored ascending in j.  Rows live column-major
// (nbr[k * N + i]) so per-row loads are contiguous across particles.  The
// half list enumerates each unordered pair once (owner i < j) with the row
// slot it occupies in both rows, so the force pass evaluates a pair once,
// writes its result into both slots, and each particle sums its own row.
//
// A build has three parts, each a grid over particles:
//   1. cells: every particle goes into the fixed-capacity slots of its cell;
//   2. rows: 16 lanes per particle scan the 3^d neighbour cells, collect
//      the hits in LDS by wave ballots, and rank-sort them into the row;
//   3. fill: each particle writes the pair entries it owns and empties its
//      cell; one workgroup recomputes the tile plan (the first tile of every
//      replica) for the pair kernel.
// The kernels here build outside a step (k_assign, k_nbr, k_fill).  Inside
// a step the same device code (dem_listbuild.h) runs in the step kernels:
// the kick-drift puts the particles into cells, extra workgroups of the
// pair kernel write the rows while the pair workgroups still use the old
// pair entries, and extra workgroups of the replica tail write the pair
// entries and the plan; the new lists serve from the next step on.
#include "dem_listbuild.h"

namespace dem {
namespace {

using lb::kNbrPer;

// Cells from the current positions (builds outside a step).
__global__ void __launch_bounds__(kBlock) k_assign(BatchParams b, const SysParams *reps, StatePtrs s, ListPtrs l,
                                                      const int64_t *budget, int mode)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = i / kChunk;
    const int r = __builtin_amdgcn_readfirstlane(c < b.nchunk ? l.chunk_rep[c] : -1);
    if (r < 0) return;
    const SysParams &p = reps[r];
    if (!lb::building(mode, r, p, l.flags + r * FLAG_COUNT, budget) || i >= p.off + p.n) return;
    if (i == p.off) l.flags[r * FLAG_COUNT + FLAG_NEWPAIRS] = 0;  // the row workgroups add the replica's pairs
    cell_insert(p, l, i, s.x[i], s.y[i], p.dim == 3 ? s.z[i] : 0.0);
}

// Neighbour rows (lb::nbr_rows), one wavefront per 4 particles.
template <int DIM>
__global__ void __launch_bounds__(64) k_nbr(BatchParams b, const SysParams *reps, StatePtrs s, ListPtrs l,
                                               const int64_t *budget, int mode)
{
    __shared__ int buf[kNbrPer * kRowMax];
    const int vb = blockIdx.x;
    const int r = l.chunk_rep[vb * kNbrPer / kChunk];
    if (r < 0) return;
    const SysParams &p = reps[r];
    int32_t *fl = l.flags + r * FLAG_COUNT;
    if (!lb::building(mode, r, p, fl, budget)) return;
    lb::nbr_rows<DIM>(b, p, s, l, fl, vb, buf);
}

// Pair offsets and entries (lb::fill_chunk), one wavefront per chunk; block
// 0 first recomputes the tile plan.
__global__ void __launch_bounds__(kBlock) k_fill(BatchParams b, const SysParams *reps, ListPtrs l,
                                                    const int64_t *budget, int mode, int clear_cells)
{
    __shared__ int part[kBlock];
    if (blockIdx.x == 0)
        lb::plan<kBlock>(b, reps, l, part, [&](int r) {
            return mode != LISTS_PLAN && mode != LISTS_REFILL &&
                   lb::building(mode, r, reps[r], l.flags + r * FLAG_COUNT, budget);
        });
    if (mode == LISTS_PLAN) return;
    const int c = (int)((blockIdx.x * blockDim.x + threadIdx.x) / kChunk);
    const int r = __builtin_amdgcn_readfirstlane(c < b.nchunk ? l.chunk_rep[c] : -1);
    if (r < 0) return;
    const SysParams &p = reps[r];
    if (!lb::building(mode, r, p, l.flags + r * FLAG_COUNT, budget)) return;
    lb::fill_chunk(b, p, l, c, mode == LISTS_REFILL, clear_cells != 0);
}

}  // namespace

void launch_lists(const Launch &L, int mode, hipStream_t stream)
{
    if (L.b.nrep == 0) return;
    const int nb = blocks_for(L.b.nchunk * kChunk);
    if (mode == LISTS_PLAN || L.b.nchunk == 0) {
        k_fill<<<1, kBlock, 0, stream>>>(L.b, L.reps, L.l, L.budget, LISTS_PLAN, 0);
        return;
    }
    if (mode == LISTS_REFILL) {
        k_fill<<<nb, kBlock, 0, stream>>>(L.b, L.reps, L.l, L.budget, LISTS_REFILL, 0);
        return;
    }
    k_assign<<<nb, kBlock, 0, stream>>>(L.b, L.reps, L.s, L.l, L.budget, mode);
    const int nbn = L.b.nchunk * (kChunk / kNbrPer);
    if (L.b.dim == 3) k_nbr<3><<<nbn, 64, 0, stream>>>(L.b, L.reps, L.s, L.l, L.budget, mode);
    else k_nbr<2><<<nbn, 64, 0, stream>>>(L.b, L.reps, L.s, L.l, L.budget, mode);
    k_fill<<<nb, kBlock, 0, stream>>>(L.b, L.reps, L.l, L.budget, mode, 1);
}

}  // namespace dem

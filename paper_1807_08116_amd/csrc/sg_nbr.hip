// sg_nbr.hip -- neighbour lists of the gas (the lists the paper's DC and HFC
// kernels build from CellSPH / indexPC / hmaxCell, Sec. 3), stored as CSR
// by sorted slot.
//
// One wavefront per target slot s.  For every non-empty level l the target
// scans the cells within R = (h_s + hmax_l)(1 + 2^-10) of itself: any pair
// passing the predicate has |r| < (h_s + h_t)(1 + 2^-20) <= R, so the scan
// is complete.  Cells with the same (level, z, y) and consecutive x are
// consecutive in key order, so each (z, y) row of the box is one contiguous
// slot range, read with coalesced loads, 64 candidates at a time; the
// bounds of up to 64 rows are fetched at once, one row per lane.  Levels
// ascend, then z, y, x, so slots come out in ascending order and rows need
// no sort.
//
// One search pass: each target writes its hits into a slot of its own,
// kSlot entries long, in a scratch array (no atomics), and counts them.  A
// scan of the counts gives the CSR offsets; a copy pass then moves every
// slot to its CSR row, and a target with more than kSlot hits (none in the
// workloads measured: at most 58) searches a second time, straight into
// its row.
//
// Built with -ffp-contract=off: the FP32 predicate must round exactly as
// specified (each product and fma rounded once).
#include "sg_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

__device__ inline unsigned rank_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// xi_ij < 2 tested in FP32: see the grid / neighbour contract in sphgrav.h.
__device__ inline bool nbr_pred(double xi, double yi, double zi, float hif, double xj, double yj,
                                double zj, double hj) {
    const float dx = (float)(xi - xj);
    const float dy = (float)(yi - yj);
    const float dz = (float)(zi - zj);
    const float dxx = dx * dx;
    const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dxx));
    const float cut = hif + (float)hj;
    const float cut2 = cut * cut;
    return r2 < cut2;
}

constexpr int64_t kSlot = 96;              // scratch entries per target

template <typename F>
__device__ inline void nbr_scan(const sg_grid_dev* __restrict__ g, int64_t ng, int64_t s,
                                unsigned lane, const double* __restrict__ xs,
                                const double* __restrict__ ys, const double* __restrict__ zs,
                                const double* __restrict__ hs, const int64_t* __restrict__ off,
                                F&& hit) {
    const double p[3] = {xs[s], ys[s], zs[s]};
    const double hi = hs[s];
    const float hif = (float)hi;
    const int nlev = g->nlev;
    for (int l = 0; l < nlev; ++l) {
        const int64_t ncell = g->ncell[l];
        if (ncell == 0) continue;
        const double R = (hi + g->hmaxlev[l]) * (1.0 + 0x1p-10);
        const double inv = g->invL[l];
        int64_t lo[3], hi3[3];
        bool empty = false;
        for (int d = 0; d < 3; ++d) {
            const double o = g->org[l][d];
            const double top = (double)(g->dim[l][d] - 1);
            double a = floor((p[d] - R - o) * inv);
            double b = floor((p[d] + R - o) * inv);
            if (b < 0.0 || a > top) empty = true;
            a = a < 0.0 ? 0.0 : (a > top ? top : a);
            b = b < 0.0 ? 0.0 : (b > top ? top : b);
            lo[d] = (int64_t)a;
            hi3[d] = (int64_t)b;
        }
        if (empty) continue;
        const int64_t base = g->base[l], dx = g->dim[l][0], dy = g->dim[l][1];
        const int64_t ny = hi3[1] - lo[1] + 1;
        const int64_t nrows = (hi3[2] - lo[2] + 1) * ny;
        for (int64_t r0 = 0; r0 < nrows; r0 += 64) {
            // bounds of rows r0 .. r0+63, one row per lane; offsets are
            // bounded by ng: clamp so that a corrupt table can never send a
            // load outside the sorted arrays
            int64_t my0 = 0, my1 = 0;
            const int64_t r = r0 + lane;
            if (r < nrows) {
                const int64_t cz = lo[2] + r / ny, cy = lo[1] + r % ny;
                const int64_t row = base + (cz * dy + cy) * dx;
                my0 = off[row + lo[0]];
                my1 = off[row + hi3[0] + 1];
                my0 = my0 < 0 ? 0 : my0;
                my1 = my1 > ng ? ng : my1;
            }
            const int nr = (int)(nrows - r0 < 64 ? nrows - r0 : 64);
            for (int k = 0; k < nr; ++k) {
                const int64_t t0 = __shfl(my0, k, 64), t1 = __shfl(my1, k, 64);
                for (int64_t tb = t0; tb < t1; tb += 64) {
                    const int64_t t = tb + lane;
                    bool ok = false;
                    if (t < t1 && t != s) ok = nbr_pred(p[0], p[1], p[2], hif, xs[t], ys[t], zs[t], hs[t]);
                    hit(__ballot(ok), t, ok);
                }
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_nbr_search(
    const sg_grid_dev* __restrict__ g, int64_t ng, const double* __restrict__ xs,
    const double* __restrict__ ys, const double* __restrict__ zs, const double* __restrict__ hs,
    const int64_t* __restrict__ off, int32_t* __restrict__ cnt, int32_t* __restrict__ slots) {
    if (g->err & SGE_SORT_FATAL) return;
    const unsigned lane = threadIdx.x & 63;
    const int64_t s = xcd_block(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6);
    if (s >= ng) return;                       // uniform per wave
    int32_t* mine = slots + s * kSlot;
    int64_t c = 0;
    nbr_scan(g, ng, s, lane, xs, ys, zs, hs, off, [&](unsigned long long mask, int64_t t, bool ok) {
        if (ok) {
            const int64_t pos = c + rank_below(mask);
            if (pos < kSlot) mine[pos] = (int32_t)t;
        }
        c += __builtin_popcountll(mask);
    });
    if (lane == 0) cnt[s] = (int32_t)c;
}

// Move every target's slot to its CSR row (or search again into the row
// when the slot was too short).
__global__ __launch_bounds__(kBlock) void k_nbr_compact(
    const sg_grid_dev* __restrict__ g, int64_t ng, const double* __restrict__ xs,
    const double* __restrict__ ys, const double* __restrict__ zs, const double* __restrict__ hs,
    const int64_t* __restrict__ off, const int32_t* __restrict__ cnt,
    const int32_t* __restrict__ slots, const int64_t* __restrict__ nbr_off,
    int32_t* __restrict__ nbr_idx) {
    if (g->err & (SGE_SORT_FATAL | SGE_NNZ)) return;
    const unsigned lane = threadIdx.x & 63;
    const int64_t s = xcd_block(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6);
    if (s >= ng) return;
    const int64_t c = cnt[s], to = nbr_off[s];
    if (c <= kSlot) {
        const int32_t* mine = slots + s * kSlot;
        for (int64_t k = lane; k < c; k += 64) nbr_idx[to + k] = mine[k];
        return;
    }
    int64_t q = 0;
    nbr_scan(g, ng, s, lane, xs, ys, zs, hs, off, [&](unsigned long long mask, int64_t t, bool ok) {
        if (ok) nbr_idx[to + q + rank_below(mask)] = (int32_t)t;
        q += __builtin_popcountll(mask);
    });
}

__global__ void k_nbr_check(sg_grid_dev* g, const int64_t* __restrict__ nbr_off, int64_t ng,
                            int64_t nnz_cap) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (g->err & SGE_SORT_FATAL) return;
    const int64_t nnz = nbr_off[ng];
    g->nnz = nnz;
    if (nnz > nnz_cap) {
        g->err |= SGE_NNZ;
        g->need_nnz = nnz;
    }
}

inline unsigned waves_grid(int64_t n) {
    int64_t b = (n + kWaves - 1) / kWaves;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

size_t sg_nbr_slot_bytes(int64_t ng) { return 4 * (size_t)kSlot * (size_t)(ng > 0 ? ng : 0); }

void sg_launch_nbr_search(const sg_grid_dev* g, int64_t ng, const double* xs, const double* ys,
                          const double* zs, const double* hs, const int64_t* off, int32_t* cnt,
                          int32_t* slots, hipStream_t st) {
    hipLaunchKernelGGL(k_nbr_search, dim3(waves_grid(ng)), dim3(kBlock), 0, st, g, ng, xs, ys, zs,
                       hs, off, cnt, slots);
}

void sg_launch_nbr_check(sg_grid_dev* g, const int64_t* nbr_off, int64_t ng, int64_t nnz_cap,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_nbr_check, dim3(1), dim3(64), 0, st, g, nbr_off, ng, nnz_cap);
}

void sg_launch_nbr_compact(const sg_grid_dev* g, int64_t ng, const double* xs, const double* ys,
                           const double* zs, const double* hs, const int64_t* off,
                           const int32_t* cnt, const int32_t* slots, const int64_t* nbr_off,
                           int32_t* nbr_idx, hipStream_t st) {
    hipLaunchKernelGGL(k_nbr_compact, dim3(waves_grid(ng)), dim3(kBlock), 0, st, g, ng, xs, ys, zs,
                       hs, off, cnt, slots, nbr_off, nbr_idx);
}

// sg_nbr.hip -- neighbour lists of the gas (the lists the paper's DC and HFC
// kernels build from CellSPH / indexPC / hmaxCell, Sec. 3), stored as CSR
// by sorted slot.
//
// One wavefront per target slot s.  For every non-empty level l the target
// scans the cells within R = (h_s + hmax_l)(1 + 2^-10) of itself: any pair
// passing the predicate has |r| < (h_s + h_t)(1 + 2^-20) <= R, so the scan
// is complete.  Cells with the same (level, z, y) and consecutive x are
// consecutive in key order, so each (z, y) row of the box is one contiguous
// slot range, read with coalesced loads, 64 candidates at a time.  Levels
// ascend, then z, y, x, so slots come out in ascending order and rows need
// no sort; count and fill passes visit candidates identically.
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

template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_nbr(const sg_grid_dev* __restrict__ g, int64_t ng,
                                                const double* __restrict__ xs,
                                                const double* __restrict__ ys,
                                                const double* __restrict__ zs,
                                                const double* __restrict__ hs,
                                                const int64_t* __restrict__ off,
                                                int32_t* __restrict__ cnt,
                                                const int64_t* __restrict__ nbr_off,
                                                int32_t* __restrict__ nbr_idx, int64_t nnz_cap) {
    const uint32_t err = g->err;
    if (err & SGE_SORT_FATAL) return;
    if (FILL && (err & SGE_NNZ)) return;
    const unsigned lane = threadIdx.x & 63;
    const int64_t s = xcd_block(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6);
    if (s >= ng) return;                       // uniform per wave
    const double p[3] = {xs[s], ys[s], zs[s]};
    const double hi = hs[s];
    const float hif = (float)hi;
    int64_t w = FILL ? nbr_off[s] : 0;
    int64_t c = 0;
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
        for (int64_t cz = lo[2]; cz <= hi3[2]; ++cz) {
            for (int64_t cy = lo[1]; cy <= hi3[1]; ++cy) {
                const int64_t row = base + (cz * dy + cy) * dx;
                // offsets are bounded by ng; clamp so that a corrupt table
                // can never send a load outside the sorted arrays
                int64_t t0 = off[row + lo[0]];
                int64_t t1 = off[row + hi3[0] + 1];
                t0 = t0 < 0 ? 0 : t0;
                t1 = t1 > ng ? ng : t1;
                for (int64_t tb = t0; tb < t1; tb += 64) {
                    const int64_t t = tb + lane;
                    bool ok = false;
                    if (t < t1 && t != s) ok = nbr_pred(p[0], p[1], p[2], hif, xs[t], ys[t], zs[t], hs[t]);
                    const unsigned long long mask = __ballot(ok);
                    if (FILL) {
                        if (ok) {
                            const int64_t pos = w + rank_below(mask);
                            if (pos < nnz_cap) nbr_idx[pos] = (int32_t)t;
                        }
                        w += __builtin_popcountll(mask);
                    } else {
                        c += __builtin_popcountll(mask);
                    }
                }
            }
        }
    }
    if (!FILL && lane == 0) cnt[s] = (int32_t)c;
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

void sg_launch_nbr_count(const sg_grid_dev* g, int64_t ng, const double* xs, const double* ys,
                         const double* zs, const double* hs, const int64_t* off, int32_t* cnt,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_nbr<false>, dim3(waves_grid(ng)), dim3(kBlock), 0, st, g, ng, xs, ys,
                       zs, hs, off, cnt, (const int64_t*)nullptr, (int32_t*)nullptr, (int64_t)0);
}

void sg_launch_nbr_check(sg_grid_dev* g, const int64_t* nbr_off, int64_t ng, int64_t nnz_cap,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_nbr_check, dim3(1), dim3(64), 0, st, g, nbr_off, ng, nnz_cap);
}

void sg_launch_nbr_fill(const sg_grid_dev* g, int64_t ng, const double* xs, const double* ys,
                        const double* zs, const double* hs, const int64_t* off,
                        const int64_t* nbr_off, int32_t* nbr_idx, int64_t nnz_cap,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_nbr<true>, dim3(waves_grid(ng)), dim3(kBlock), 0, st, g, ng, xs, ys,
                       zs, hs, off, (int32_t*)nullptr, nbr_off, nbr_idx, nnz_cap);
}

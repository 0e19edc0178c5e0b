// sg_nbr.hip -- neighbour lists of the gas (the lists the paper's DC and HFC
// kernels build from CellSPH / indexPC / hmaxCell, Sec. 3), stored as CSR
// by sorted slot.
//
// Search region.  For every non-empty level l a target s must scan the
// cells within R = (h_s + hmax_l)(1 + 2^-10) of itself: any pair passing
// the predicate has |r| < (h_s + h_t)(1 + 2^-20) <= R, so the scan is
// complete.  Cells with the same (level, z, y) and consecutive x are
// consecutive in key order, so each (z, y) row of a box of cells is one
// contiguous slot range, and visiting levels, then z, y, x in ascending
// order yields candidates in ascending slot order: rows need no sort.
//
// Cell-staged search (k_nbr_search).  One wavefront takes 32 consecutive
// target slots and walks them cell by cell: the targets that share a cell
// key form a run, and the run's search region is the union (per level) of
// its targets' boxes.  The rows of that region are flattened into one
// candidate stream, loaded 192 candidates at a time (three per lane) and
// held in registers while every target of the run tests them, so a
// candidate is fetched once per cell instead of once per target.  Any
// grouping gives the same lists: the union contains each target's own box,
// and every target keeps only the candidates that pass its predicate, in
// stream order.  The union box is a pair of DPP reductions per dimension,
// the stream offsets a DPP scan of the row lengths, and each batch of 64
// stream positions finds its slots by walking the few non-empty rows that
// overlap it: the set-up makes no LDS round trips.
//
// Each target writes its hits into a slot of its own, kSlot entries long,
// in a scratch array (no atomics), and counts them.  A scan of the counts
// gives the CSR offsets; a copy pass then moves every slot to its CSR row,
// and a target with more than kSlot hits (none in the collision workloads:
// at most 58 at 2M particles; clustered gas can have thousands) searches a
// second time, alone, straight into its row.
//
// Built with -ffp-contract=off: the FP32 predicate must round exactly as
// specified (each product and fma rounded once).
#include "sg_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
// Targets per wavefront of the search (lanes 0 .. kTargets-1 hold them;
// all 64 lanes hold candidates).  The search is bound by the vector-ALU
// work of its pair tests (busy 85 % of the kernel at 2M particles),
// and the wavefronts' work varies widely (runs of 1 to 64 targets, union
// boxes over 1 to 5 levels), so shorter wavefronts pack the SIMDs better
// at the end of the launch: the search stage took 1.62 ms with 64 targets
// per wavefront, 1.53 ms with 32 and 1.57 ms with 16 (each run cut at a
// wavefront boundary repeats its boxes' setup and candidate loads); with
// the set-up as it is now, 0.98-0.99, 0.96-0.97 and 1.00 ms.
constexpr int kTargets = 32;
// Candidate batches held in registers per target pass: each target's data
// is read and its hit count fetched once per kHold batches instead of once
// per batch.  Search stage at 2M particles when the target data were lane
// reads (about 23 instead of 28 vector instructions per 64 pair tests):
// 1.53 ms with one batch, 1.41 with 2, 1.32 with 4, 1.49 with 8 (113 VGPRs:
// 4 waves per SIMD).  With the set-up as it is now: 2: 0.98-0.99 ms, 3:
// 0.94 (63 VGPRs), 4: 0.96, 6: 1.01-1.02.
constexpr int kHold = 3;

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

// The same predicate with the candidate's h already rounded to FP32.
__device__ inline bool nbr_pred_f(double xi, double yi, double zi, float hif, double xj,
                                  double yj, double zj, float hjf) {
    const float dx = (float)(xi - xj);
    const float dy = (float)(yi - yj);
    const float dz = (float)(zi - zj);
    const float dxx = dx * dx;
    const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dxx));
    const float cut = hif + hjf;
    const float cut2 = cut * cut;
    return r2 < cut2;
}

constexpr int64_t kSlot = 96;              // scratch entries per target

// Cells [lo, hi] (per dimension, clamped to the grid) of level l within
// R = (h + hmax_l)(1 + 2^-10) of p; false when the level has no such cell.
__device__ inline bool level_box(const sg_grid_dev* __restrict__ g, int l, const double p[3],
                                 double h, int32_t lo[3], int32_t hi3[3]) {
    // in cell units: the reach R inv and the position (p - o) inv (their
    // rounding differs from that of (p +- R - o) inv by far less than the
    // 2^-10 margin of R, so the box still holds every cell within reach)
    const double inv = g->invL[l];
    const double Ri = (h + g->hmaxlev[l]) * (1.0 + 0x1p-10) * inv;
    bool empty = false;
    for (int d = 0; d < 3; ++d) {
        const double c = (p[d] - g->org[l][d]) * inv;
        // clamped into [-1, 2^30] first, where the conversion is exact (a
        // NaN becomes -1: an empty box)
        const int32_t a = (int32_t)fmin(fmax(floor(c - Ri), -1.0), 0x1p30);
        const int32_t b = (int32_t)fmin(fmax(floor(c + Ri), -1.0), 0x1p30);
        const int32_t top = (int32_t)g->dim[l][d] - 1;
        if (b < 0 || a > top) empty = true;
        lo[d] = min(max(a, 0), top);
        hi3[d] = min(max(b, 0), top);
    }
    return !empty;
}

// One target's scan over its own boxes (used by the overflow path).
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
        if (g->ncell[l] == 0) continue;
        int32_t lo[3], hi3[3];
        if (!level_box(g, l, p, hi, lo, hi3)) continue;
        const int64_t base = g->base[l], dx = g->dim[l][0], dy = g->dim[l][1];
        const int64_t ny = (int64_t)hi3[1] - lo[1] + 1;
        const int64_t nrows = ((int64_t)hi3[2] - lo[2] + 1) * ny;
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

// Cross-lane reductions and scan by DPP row operations (no LDS round
// trips; every lane of the wavefront must be active).  Controls:
// quad_perm [1,0,3,2] 0xb1, [2,3,0,1] 0x4e, row_shr:n 0x110 + n,
// row_mirror 0x140, row_half_mirror 0x141, row_bcast:15 0x142 (lane 15 of
// each row into the next row), row_bcast:31 0x143 (lane 31 into rows 2, 3).
template <int kCtrl, int kRowMask = 0xf>
__device__ inline int32_t dpp(int32_t old, int32_t v) {
    return __builtin_amdgcn_update_dpp(old, v, kCtrl, kRowMask, 0xf, false);
}

// minimum over the 64 lanes (uniform result)
__device__ inline int32_t wave_min(int32_t v) {
    constexpr int32_t I = INT32_MAX;
    v = min(v, dpp<0xb1>(I, v));
    v = min(v, dpp<0x4e>(I, v));
    v = min(v, dpp<0x141>(I, v));
    v = min(v, dpp<0x140>(I, v));              // each row of 16: its minimum
    v = min(v, dpp<0x142, 0xa>(I, v));         // rows 1, 3: with rows 0, 2
    v = min(v, dpp<0x143, 0xc>(I, v));         // rows 2, 3: with rows 0, 1
    return __builtin_amdgcn_readlane(v, 63);
}

// maximum over the 64 lanes (uniform result)
__device__ inline int32_t wave_max(int32_t v) {
    constexpr int32_t I = INT32_MIN;
    v = max(v, dpp<0xb1>(I, v));
    v = max(v, dpp<0x4e>(I, v));
    v = max(v, dpp<0x141>(I, v));
    v = max(v, dpp<0x140>(I, v));
    v = max(v, dpp<0x142, 0xa>(I, v));
    v = max(v, dpp<0x143, 0xc>(I, v));
    return __builtin_amdgcn_readlane(v, 63);
}

// inclusive prefix sum over the 64 lanes
__device__ inline int32_t wave_incl_sum(int32_t v) {
    v += dpp<0x111>(0, v);                     // within each row of 16
    v += dpp<0x112>(0, v);
    v += dpp<0x114>(0, v);
    v += dpp<0x118>(0, v);
    v += dpp<0x142, 0xa>(0, v);                // rows 1, 3: + total of rows 0, 2
    v += dpp<0x143, 0xc>(0, v);                // rows 2, 3: + total of rows 0, 1
    return v;
}

// The search of wavefront w (target slots kTargets w onward); w is uniform.
__device__ __attribute__((always_inline)) inline void nbr_search_wave(
    const sg_grid_dev* __restrict__ g, int64_t ng, const double* __restrict__ xs,
    const double* __restrict__ ys, const double* __restrict__ zs, const double* __restrict__ hs,
    const int64_t* __restrict__ off, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ key, int32_t* __restrict__ cnt, int32_t* __restrict__ slots,
    int32_t w) {
    if (g->err & SGE_SORT_FATAL) return;
    const unsigned lane = threadIdx.x & 63;
    const int64_t g0 = (int64_t)w * kTargets;
    if (g0 >= ng) return;
    const int64_t s = g0 + lane;
    const bool live = lane < (unsigned)kTargets && s < ng;
    double p[3] = {0.0, 0.0, 0.0}, h = 0.0;
    int32_t k = -1;
    if (live) {
        p[0] = xs[s];
        p[1] = ys[s];
        p[2] = zs[s];
        h = hs[s];
        const int32_t i = perm[s];
        // the key only groups targets (any grouping is correct)
        k = (uint32_t)i < (uint64_t)ng ? key[i] : -2 - (int32_t)lane;
    }
    const float hif = (float)h;
    // the wavefront's targets in LDS: a target pass reads its target's
    // record with broadcast loads (one address instruction) instead of
    // seven lane reads on the vector ALU (search stage at 1M gas 1.147 ->
    // 1.096 ms); 4 KB per workgroup, which still fits beside the gravity
    // kernel's workgroups on a compute unit
    struct target_rec { double x, y, z; float h, pad; };
    __shared__ target_rec tp[kWaves][kTargets];
    target_rec* const mytp = tp[threadIdx.x >> 6];
    if (lane < (unsigned)kTargets) mytp[lane] = target_rec{p[0], p[1], p[2], hif, 0.0f};
    __builtin_amdgcn_wave_barrier();
    int32_t mine = 0;                          // hits of target g0 + lane so far
    const int nlev = g->nlev;
    unsigned long long todo = __ballot(live);
    while (todo) {
        const int lead = __builtin_ctzll(todo);
        const int32_t rk = __builtin_amdgcn_readlane(k, lead);
        const unsigned long long run = __ballot(live && k == rk) & todo;
        todo &= ~run;
        const bool inrun = (run >> lane) & 1ull;
        for (int l = 0; l < nlev; ++l) {
            if (g->ncell[l] == 0) continue;
            int32_t lo[3], hi3[3];
            const bool has = inrun && level_box(g, l, p, h, lo, hi3);
            // no target of the run reaches level l: skipped before the
            // reductions (search stage at 1M gas 1.015 -> 0.96-0.97 ms)
            if (__ballot(has) == 0ull) continue;
            // union of the run's boxes; wave-uniform, held in scalar
            // registers so that every loop below is uniform and its
            // cross-lane reads see all lanes
            int32_t ulo[3], uhi[3];
            bool inside = true;
            for (int d = 0; d < 3; ++d) {
                ulo[d] = wave_min(has ? lo[d] : INT32_MAX);
                uhi[d] = wave_max(has ? hi3[d] : -1);
                inside = inside && ulo[d] >= 0 && ulo[d] <= uhi[d] && uhi[d] < g->dim[l][d];
            }
            // no target of the run reaches level l (the box test also
            // keeps every row and cell index below inside the level)
            if (!inside) continue;
            const int64_t base = g->base[l];
            const int32_t dx = (int32_t)g->dim[l][0], dy = (int32_t)g->dim[l][1];
            const uint32_t ny = (uint32_t)(uhi[1] - ulo[1] + 1);
            const int32_t nrows = (int32_t)((uint32_t)(uhi[2] - ulo[2] + 1) * ny);
            for (int32_t r0 = 0; r0 < nrows; r0 += 64) {
                // rows r0 .. r0+63, one per lane: first slot and length
                // (offsets clamped to [0, ng] so that a corrupt table can
                // never send a load outside the sorted arrays); row and
                // cell indices fit int32 (a level's cell count does)
                int32_t first = 0, len = 0;
                const int32_t r = r0 + (int32_t)lane;
                if (r < nrows) {
                    const uint32_t rz = (uint32_t)r / ny;
                    const int32_t cz = ulo[2] + (int32_t)rz, cy = ulo[1] + (int32_t)((uint32_t)r - rz * ny);
                    const int64_t row = base + (int64_t)((cz * dy + cy) * dx);
                    int64_t a = off[row + ulo[0]], b = off[row + uhi[0] + 1];
                    a = a < 0 ? 0 : (a > ng ? ng : a);
                    b = b < a ? a : (b > ng ? ng : b);
                    first = (int32_t)a;
                    len = (int32_t)(b - a);
                }
                // flatten: the rows are disjoint slot ranges, so the total
                // is at most ng
                const int32_t incl = wave_incl_sum(len);
                const int32_t start = incl - len;
                const int32_t total = __builtin_amdgcn_readlane(incl, 63);
                // stream positions b .. b+63 -> slots, one per lane: of the
                // non-empty rows that overlap them (a few; ascending, each
                // starting where the previous one ends) each lane keeps the
                // last one that starts at or before its position
                const int32_t fs = first - start;
                auto locate = [&](int32_t b) -> int32_t {
                    const int32_t q = b + (int32_t)lane;
                    int32_t d = 0;
                    for (unsigned long long m = __ballot(len > 0 && start < b + 64 && incl > b); m;
                         m &= m - 1) {
                        const int j = __builtin_ctzll(m);
                        const int32_t sj = __builtin_amdgcn_readlane(start, j);
                        const int32_t dj = __builtin_amdgcn_readlane(fs, j);
                        if (q >= sj) d = dj;
                    }
                    return q + d;
                };
                // candidates in chunks of kHold batches of 64, held in
                // registers while each target of the run tests the whole
                // chunk (its record read from LDS once per chunk, its hit
                // count carried in a scalar register)
                for (int32_t cb0 = 0; cb0 < total; cb0 += 64 * kHold) {
                    int32_t tk[kHold];
                    bool vk[kHold];
                    unsigned long long vm[kHold];          // lanes holding a candidate
                    double xk[kHold], yk[kHold], zk[kHold];
                    float hk[kHold];
                    // every batch's loads are issued before any is used
                    // (h converts to FP32 after the last one); lanes past
                    // the stream load a clamped slot and are masked out
                    double hd[kHold];
#pragma unroll
                    for (int k = 0; k < kHold; ++k) {
                        const int32_t q = cb0 + 64 * k + (int32_t)lane;
                        vk[k] = q < total;
                        tk[k] = 0;
                        xk[k] = yk[k] = zk[k] = hd[k] = 0.0;
                        if (cb0 + 64 * k < total) {          // uniform
                            tk[k] = locate(cb0 + 64 * k);
                            const int32_t t = min(max(tk[k], 0), (int32_t)(ng - 1));
                            xk[k] = xs[t];
                            yk[k] = ys[t];
                            zk[k] = zs[t];
                            hd[k] = hs[t];
                        }
                        const int32_t nk = total - (cb0 + 64 * k);
                        vm[k] = nk >= 64 ? ~0ull : (nk > 0 ? (1ull << nk) - 1 : 0ull);
                    }
                    // (an empty statement that takes the loaded values keeps
                    // the conversions, and their waits, behind the last load)
                    static_assert(kHold == 3, "the statement below names each held batch");
                    asm volatile("" : "+v"(hd[0]), "+v"(hd[1]), "+v"(hd[2]));
#pragma unroll
                    for (int k = 0; k < kHold; ++k) hk[k] = (float)hd[k];
                    for (unsigned long long tr = run; tr; tr &= tr - 1) {
                        const int L = __builtin_ctzll(tr);
                        const int64_t sL = g0 + L;
                        // target L's data (uniform)
                        const double xi = mytp[L].x, yi = mytp[L].y, zi = mytp[L].z;
                        const float hi = mytp[L].h;
                        int32_t c = __builtin_amdgcn_readlane(mine, L);
                        int32_t* const row = slots + sL * kSlot;
#pragma unroll
                        for (int k = 0; k < kHold; ++k) {
                            if (cb0 + 64 * k >= total) break;  // uniform
                            // the ballot of the bare comparison is the
                            // comparison's own lane mask and validity a
                            // scalar mask; the target itself is looked for
                            // only in batches with a hit
                            const bool pr = nbr_pred_f(xi, yi, zi, hi, xk[k], yk[k], zk[k], hk[k]);
                            unsigned long long mask = __builtin_amdgcn_ballot_w64(pr) & vm[k];
                            if (mask) {
                                const bool me = tk[k] == (int32_t)sL;
                                mask &= ~__builtin_amdgcn_ballot_w64(me);
                                const uint32_t pos = (uint32_t)c + (uint32_t)rank_below(mask);
                                if (pr && vk[k] && !me && pos < (uint32_t)kSlot) row[pos] = tk[k];
                                c += __builtin_popcountll(mask);
                            }
                        }
                        // lane L's count := c (one lane written, whatever the
                        // execution mask)
                        asm volatile("v_writelane_b32 %0, %1, m0" : "+v"(mine) : "s"(c), "{m0}"(L));
                    }
                }
            }
        }
    }
    if (live) cnt[s] = mine;
}

__global__ __launch_bounds__(kBlock) void k_nbr_search(
    const sg_grid_dev* __restrict__ g, int64_t ng, const double* __restrict__ xs,
    const double* __restrict__ ys, const double* __restrict__ zs, const double* __restrict__ hs,
    const int64_t* __restrict__ off, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ key, int32_t* __restrict__ cnt, int32_t* __restrict__ slots) {
    // first target slot of this wavefront (uniform: held in a scalar
    // register).  The XCDs take chunks of 16 consecutive workgroups in
    // turn: the work per slot varies across the collision, and handing
    // each XCD one contiguous share of the slots left some XCDs busy after
    // the others had drained (stage 1.83 -> 1.64 ms at 1M gas), while
    // plain launch order spreads neighbouring targets over all 8 L2s
    // (1.5x the fetched bytes of chunks of 16, at the same time).
    const int32_t w = __builtin_amdgcn_readfirstlane(
        (int32_t)(xcd_chunk_block(blockIdx.x, gridDim.x, 16) * kWaves + (threadIdx.x >> 6)));
    nbr_search_wave(g, ng, xs, ys, zs, hs, off, perm, key, cnt, slots, w);
}

// Move every target's slot to its CSR row (or search again into the row
// when the slot was too short).  Wavefront w takes targets
// kCompact w .. kCompact w + kCompact - 1, 64 / kCompact lanes each; a target
// with more than kSlot hits is searched again by the whole wavefront.
// Targets per wavefront at 1M gas (about 41 hits each), neighbour stage:
// 2: 1.23 ms, 4: 1.17-1.19, 8: 1.14-1.16, 16: 1.18, 32: 1.31.
constexpr int kCompact = 8;
constexpr int kCompactLanes = 64 / kCompact;

__device__ __attribute__((always_inline)) inline void nbr_compact_wave(
    const sg_grid_dev* __restrict__ g, int64_t ng, const double* __restrict__ xs,
    const double* __restrict__ ys, const double* __restrict__ zs, const double* __restrict__ hs,
    const int64_t* __restrict__ off, const int32_t* __restrict__ cnt,
    const int32_t* __restrict__ slots, const int64_t* __restrict__ nbr_off,
    int32_t* __restrict__ nbr_idx, int64_t w) {
    if (g->err & (SGE_SORT_FATAL | SGE_NNZ)) return;
    const unsigned lane = threadIdx.x & 63;
    const int64_t s0 = w * kCompact;
    if (s0 >= ng) return;
    const int64_t s = s0 + lane / kCompactLanes;
    const int64_t c = s < ng ? cnt[s] : 0;
    if (c <= kSlot) {
        const int32_t* mine = slots + s * kSlot;
        const int64_t to = nbr_off[s < ng ? s : 0];
        // four entries in flight per lane, then the rest
        int64_t k = lane % kCompactLanes;
        for (; k + 3 * kCompactLanes < c; k += 4 * kCompactLanes) {
            const int32_t v0 = mine[k], v1 = mine[k + kCompactLanes];
            const int32_t v2 = mine[k + 2 * kCompactLanes], v3 = mine[k + 3 * kCompactLanes];
            nbr_idx[to + k] = v0;
            nbr_idx[to + k + kCompactLanes] = v1;
            nbr_idx[to + k + 2 * kCompactLanes] = v2;
            nbr_idx[to + k + 3 * kCompactLanes] = v3;
        }
        for (; k < c; k += kCompactLanes) nbr_idx[to + k] = mine[k];
    }
    for (int j = 0; j < kCompact; ++j) {
        const int64_t sj = s0 + j;
        if (sj >= ng) break;
        const int64_t to = nbr_off[sj];
        if (cnt[sj] <= kSlot) continue;
        int64_t q = 0;
        nbr_scan(g, ng, sj, lane, xs, ys, zs, hs, off,
                 [&](unsigned long long mask, int64_t t, bool ok) {
                     if (ok) nbr_idx[to + q + rank_below(mask)] = (int32_t)t;
                     q += __builtin_popcountll(mask);
                 });
    }
}

__global__ __launch_bounds__(kBlock) void k_nbr_compact(
    const sg_grid_dev* __restrict__ g, int64_t ng, const double* __restrict__ xs,
    const double* __restrict__ ys, const double* __restrict__ zs, const double* __restrict__ hs,
    const int64_t* __restrict__ off, const int32_t* __restrict__ cnt,
    const int32_t* __restrict__ slots, const int64_t* __restrict__ nbr_off,
    int32_t* __restrict__ nbr_idx) {
    const int64_t w = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    nbr_compact_wave(g, ng, xs, ys, zs, hs, off, cnt, slots, nbr_off, nbr_idx, w);
}

__device__ inline void nbr_check_one(sg_grid_dev* g, const int64_t* __restrict__ nbr_off,
                                     int64_t ng, int64_t nnz_cap) {
    if (g->err & SGE_SORT_FATAL) return;
    const int64_t nnz = nbr_off[ng];
    g->nnz = nnz;
    if (nnz > nnz_cap) {
        atomicOr(&g->err, SGE_NNZ);
        g->need_nnz = nnz;
    }
}

__global__ void k_nbr_check(sg_grid_dev* g, const int64_t* __restrict__ nbr_off, int64_t ng,
                            int64_t nnz_cap) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    nbr_check_one(g, nbr_off, ng, nnz_cap);
}

// ----------------------------------------------------- all systems at once --
// (see sg_seg in sg_internal.h)

__global__ __launch_bounds__(kBlock) void k_seg_nbr_search(const sg_seg_sys* __restrict__ sys,
                                                           const int64_t* __restrict__ pfx,
                                                           int nsys) {
    int64_t lb;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &lb)];
    const int32_t w = __builtin_amdgcn_readfirstlane((int32_t)(lb * kWaves + (threadIdx.x >> 6)));
    const sg_sph_bufs& b = S.sph;
    nbr_search_wave(S.g, S.ng, b.xs, b.ys, b.zs, b.hs, S.off, b.perm, S.key, S.ncnt, S.slots, w);
}

__global__ void k_seg_nbr_check(const sg_seg_sys* __restrict__ sys, int nsys) {
    for (int k = threadIdx.x; k < nsys; k += blockDim.x)
        if (sys[k].ng > 0) nbr_check_one(sys[k].g, sys[k].sph.nbr_off, sys[k].ng, sys[k].nnz_cap);
}

__global__ __launch_bounds__(kBlock) void k_seg_nbr_compact(const sg_seg_sys* __restrict__ sys,
                                                            const int64_t* __restrict__ pfx,
                                                            int nsys) {
    int64_t lb;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &lb)];
    const sg_sph_bufs& b = S.sph;
    nbr_compact_wave(S.g, S.ng, b.xs, b.ys, b.zs, b.hs, S.off, S.ncnt, S.slots, b.nbr_off,
                     const_cast<int32_t*>(b.nbr_idx), lb * kWaves + (threadIdx.x >> 6));
}

inline unsigned waves_grid(int64_t n) {
    int64_t b = (n + kWaves - 1) / kWaves;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

void sg_seg_launch_nbr_search(const sg_seg& s, hipStream_t st) {
    if (s.nblk[SG_SEG_NBR] > 0)
        hipLaunchKernelGGL(k_seg_nbr_search, dim3((unsigned)s.nblk[SG_SEG_NBR]), dim3(kBlock), 0, st,
                           s.sys, s.pfx + SG_SEG_NBR * (s.nsys + 1), s.nsys);
}

void sg_seg_launch_nbr_finish(const sg_seg& s, hipStream_t st) {
    if (s.nblk[SG_SEG_CPT] == 0) return;
    hipLaunchKernelGGL(k_seg_nbr_check, dim3(1), dim3(64), 0, st, s.sys, s.nsys);
    hipLaunchKernelGGL(k_seg_nbr_compact, dim3((unsigned)s.nblk[SG_SEG_CPT]), dim3(kBlock), 0, st,
                       s.sys, s.pfx + SG_SEG_CPT * (s.nsys + 1), s.nsys);
}

int64_t sg_compact_blocks(int64_t ng) {
    const int64_t per = (int64_t)kWaves * kCompact;
    return (ng + per - 1) / per;
}

int64_t sg_nbr_blocks(int64_t ng) {
    const int64_t per = (int64_t)kWaves * kTargets;
    return (ng + per - 1) / per;
}

size_t sg_nbr_slot_bytes(int64_t ng) { return 4 * (size_t)kSlot * (size_t)(ng > 0 ? ng : 0); }

void sg_launch_nbr_search(const sg_grid_dev* g, int64_t ng, const double* xs, const double* ys,
                          const double* zs, const double* hs, const int64_t* off,
                          const int32_t* perm, const int32_t* key, int32_t* cnt, int32_t* slots,
                          hipStream_t st) {
    // one wavefront per kTargets target slots
    hipLaunchKernelGGL(k_nbr_search, dim3(waves_grid((ng + kTargets - 1) / kTargets)), dim3(kBlock), 0, st, g, ng,
                       xs, ys, zs, hs, off, perm, key, cnt, slots);
}

void sg_launch_nbr_check(sg_grid_dev* g, const int64_t* nbr_off, int64_t ng, int64_t nnz_cap,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_nbr_check, dim3(1), dim3(64), 0, st, g, nbr_off, ng, nnz_cap);
}

void sg_launch_nbr_compact(const sg_grid_dev* g, int64_t ng, const double* xs, const double* ys,
                           const double* zs, const double* hs, const int64_t* off,
                           const int32_t* cnt, const int32_t* slots, const int64_t* nbr_off,
                           int32_t* nbr_idx, hipStream_t st) {
    hipLaunchKernelGGL(k_nbr_compact, dim3(waves_grid((ng + kCompact - 1) / kCompact)), dim3(kBlock),
                       0, st, g, ng, xs, ys, zs,
                       hs, off, cnt, slots, nbr_off, nbr_idx);
}

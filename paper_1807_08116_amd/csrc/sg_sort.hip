// sg_sort.hip -- grid sorting of the gas (the SP kernel set of Sec. 3):
// smoothing-length levels and grid parameters, cell keys, per-cell counts
// and maximum h, prefix sums for cell offsets, stable reorder and gather of
// the sorted state.  Also the generic scan used for cell and CSR offsets,
// and a stable LSD radix sort producing a Morton order of all particles.
//
// Built with -ffp-contract=off: the key arithmetic must round exactly like
// the plain FP64 definition of the grid.
#include "sg_internal.h"

namespace {

constexpr int kBlock = 256;

__device__ inline unsigned lane_id() { return threadIdx.x & 63; }

// 64-bit minimum and maximum over the 64 lanes by DPP row operations on the
// two 32-bit halves, with no chain of shuffles through LDS (h minimum,
// Morton box, equal-key runs of the key pass).  Every lane must be active;
// the result is uniform.  Controls: quad_perm
// [1,0,3,2] 0xb1, [2,3,0,1] 0x4e, row_half_mirror 0x141, row_mirror 0x140,
// row_bcast:15 0x142 (lane 15 of each row into the next row), row_bcast:31
// 0x143 (lane 31 into rows 2 and 3).
template <int kCtrl, int kRowMask = 0xf>
__device__ inline unsigned long long dpp_u64(unsigned long long old, unsigned long long v) {
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)old, (int)(unsigned)v,
                                                              kCtrl, kRowMask, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(
        (int)(unsigned)(old >> 32), (int)(unsigned)(v >> 32), kCtrl, kRowMask, 0xf, false);
    return ((unsigned long long)hi << 32) | lo;
}
template <bool kMax>
__device__ inline unsigned long long wave_ext_u64(unsigned long long v) {
    constexpr unsigned long long I = kMax ? 0ull : ~0ull;
    auto pick = [](unsigned long long a, unsigned long long b) { return (kMax ? b > a : b < a) ? b : a; };
    v = pick(v, dpp_u64<0xb1>(I, v));
    v = pick(v, dpp_u64<0x4e>(I, v));
    v = pick(v, dpp_u64<0x141>(I, v));
    v = pick(v, dpp_u64<0x140>(I, v));          // each row of 16: its extreme
    v = pick(v, dpp_u64<0x142, 0xa>(I, v));     // rows 1, 3: with rows 0, 2
    v = pick(v, dpp_u64<0x143, 0xc>(I, v));     // rows 2, 3: with rows 0, 1
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}
__device__ inline unsigned long long wave_min_u64(unsigned long long v) { return wave_ext_u64<false>(v); }
__device__ inline unsigned long long wave_max_u64(unsigned long long v) { return wave_ext_u64<true>(v); }
__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// Number of set bits of `mask` below this lane.
__device__ inline unsigned rank_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// ------------------------------------------------------------------ scan --
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ inline int64_t scan_n(int64_t n_host, const int64_t* n_dev, int64_t cap) {
    const int64_t n = n_dev ? *n_dev : n_host;
    return n < cap ? n : cap;
}

__device__ inline void scan_reduce_tile(const int32_t* __restrict__ in, int64_t n, int64_t tile,
                                        int64_t* __restrict__ bsum) {
    const int64_t base = tile * kScanTile;
    int64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k * kBlock + threadIdx.x;
        if (i < n) s += in[i];
    }
    s = (int64_t)wave_sum_u64((unsigned long long)s);
    __shared__ int64_t ws[kBlock / 64];
    if (lane_id() == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < kBlock / 64; ++w) t += ws[w];
        bsum[tile] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const int32_t* __restrict__ in,
                                                        int64_t n_host,
                                                        const int64_t* __restrict__ n_dev,
                                                        int64_t cap,
                                                        int64_t* __restrict__ bsum) {
    scan_reduce_tile(in, scan_n(n_host, n_dev, cap), blockIdx.x, bsum);
}

// Exclusive scan of the block sums in place; out[n] = total.  256 threads,
// 4 sums each per pass: one wavefront per SIMD, so the block also finds
// room on CUs that another kernel's workgroups mostly fill.
__device__ inline void scan_bsums_block(int64_t* __restrict__ bsum, int64_t n,
                                        int64_t* __restrict__ out) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    __shared__ int64_t buf[256];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
        const int64_t i0 = c0 + 4 * (int64_t)threadIdx.x;
        int64_t v[4];
        int64_t tsum = 0;
        for (int k = 0; k < 4; ++k) {
            v[k] = i0 + k < nb ? bsum[i0 + k] : 0;
            tsum += v[k];
        }
        buf[threadIdx.x] = tsum;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {       // Hillis-Steele inclusive scan
            int64_t t = threadIdx.x >= (unsigned)o ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        int64_t run = carry + buf[threadIdx.x] - tsum;
        for (int k = 0; k < 4; ++k) {
            if (i0 + k < nb) bsum[i0 + k] = run;
            run += v[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) carry += buf[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = carry;
}

__global__ __launch_bounds__(256) void k_scan_bsums(int64_t* __restrict__ bsum, int64_t n_host,
                                                    const int64_t* __restrict__ n_dev,
                                                    int64_t cap, int64_t* __restrict__ out) {
    scan_bsums_block(bsum, scan_n(n_host, n_dev, cap), out);
}

__device__ inline void scan_down_tile(const int32_t* __restrict__ in, int64_t* __restrict__ out,
                                      int64_t n, int64_t tile,
                                      const int64_t* __restrict__ bsum) {
    const int64_t base = tile * kScanTile;
    if (base >= n) return;
    const int64_t i0 = base + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t tsum = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (i0 + k < n) ? in[i0 + k] : 0;
        tsum += v[k];
    }
    // exclusive scan of the thread sums across the block
    int64_t incl = tsum;
    for (int o = 1; o < 64; o <<= 1) {
        int64_t t = __shfl_up(incl, o, 64);
        if (lane_id() >= (unsigned)o) incl += t;
    }
    __shared__ int64_t wtot[kBlock / 64];
    if (lane_id() == 63) wtot[threadIdx.x >> 6] = incl;
    __syncthreads();
    int64_t wbase = 0;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) wbase += wtot[w];
    int64_t run = bsum[tile] + wbase + incl - tsum;
    for (int k = 0; k < kScanItems; ++k) {
        if (i0 + k < n) out[i0 + k] = run;
        run += v[k];
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_down(const int32_t* __restrict__ in,
                                                      int64_t* __restrict__ out, int64_t n_host,
                                                      const int64_t* __restrict__ n_dev,
                                                      int64_t cap,
                                                      const int64_t* __restrict__ bsum) {
    scan_down_tile(in, out, scan_n(n_host, n_dev, cap), blockIdx.x, bsum);
}

// ------------------------------------------------------------ grid rule --

__device__ inline bool finite_d(double v) { return __builtin_isfinite(v); }

// Smallest power of two >= t (t positive and normal).
__device__ inline double pow2_ceil(double t) {
    unsigned long long b = (unsigned long long)__builtin_bit_cast(long long, t);
    unsigned long long mant = b & 0x000fffffffffffffull;
    if (mant == 0) return t;
    unsigned long long e = (b >> 52) & 0x7ff;
    return __builtin_bit_cast(double, (long long)((e + 1) << 52));
}

// First level l with L0 * 2^l >= h (2 + 2^-9); -1 beyond SG_MAXLEV.
__device__ inline int level_of(double h, double L0) {
    double t = h * (2.0 + 0x1p-9);
    double L = L0;
    int l = 0;
    while (L < t) {
        L *= 2.0;
        if (++l >= SG_MAXLEV) return -1;
    }
    return l;
}

__global__ void k_status_clear(sg_grid_dev* g) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        g->err = 0;
        g->need_cells = 0;
        g->need_nnz = 0;
    }
}

__device__ inline void grid_reset_one(sg_grid_dev* g) {
    int t = threadIdx.x;
    if (t == 0) {
        g->hmin_bits = ~0ull;
        g->nnz = 0;
        g->M = 0;
        g->nlev = 0;
    }
    if (t < SG_MAXLEV) {
        for (int d = 0; d < 3; ++d) {
            g->lo[t][d] = ~0ull;
            g->hi[t][d] = 0ull;
        }
        g->hmax_bits[t] = 0ull;
        g->npart[t] = 0ull;
        g->ncell[t] = 0;
    }
    // glo / ghi belong to the gravity preparation, which resets them itself
}

__global__ void k_grid_reset(sg_grid_dev* g) { grid_reset_one(g); }

// Minimum h and validity of the gas state: a thread's items, then the
// wavefront and workgroup minimum, one global atomic per workgroup.
__device__ inline void hmin_item(const double* __restrict__ x, const double* __restrict__ y,
                                 const double* __restrict__ z, const double* __restrict__ h,
                                 int64_t i, unsigned long long& mn, bool& bad) {
    double hi = h[i];
    if (!(hi > 0.0) || !finite_d(hi) || !finite_d(x[i]) || !finite_d(y[i]) || !finite_d(z[i]))
        bad = true;
    else {
        unsigned long long o = sg_ord(hi);
        mn = o < mn ? o : mn;
    }
}

__device__ inline void hmin_fold(unsigned long long mn, bool bad, sg_grid_dev* g) {
    __shared__ unsigned long long s_mn[kBlock / 64];
    mn = wave_min_u64(mn);
    if (lane_id() == 0) s_mn[threadIdx.x >> 6] = mn;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kBlock / 64; ++k) mn = s_mn[k] < mn ? s_mn[k] : mn;
        if (mn != ~0ull) atomicMin(&g->hmin_bits, mn);
    }
    if (bad) atomicOr(&g->err, SGE_NONFINITE);
}

__global__ __launch_bounds__(kBlock) void k_grid_hmin(const double* __restrict__ x,
                                                      const double* __restrict__ y,
                                                      const double* __restrict__ z,
                                                      const double* __restrict__ h, int64_t ng,
                                                      sg_grid_dev* g) {
    unsigned long long mn = ~0ull;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < ng;
         i += (int64_t)gridDim.x * kBlock)
        hmin_item(x, y, z, h, i, mn, bad);
    hmin_fold(mn, bad, g);
}

// Per-level bounding boxes, maximum h and particle counts.
// Items base + r * stride + threadIdx.x, r < nround, of a workgroup.
__device__ inline void grid_levels_block(const double* __restrict__ x,
                                         const double* __restrict__ y,
                                         const double* __restrict__ z,
                                         const double* __restrict__ h, int64_t ng,
                                         sg_grid_dev* g, int64_t base, int64_t stride,
                                         int64_t nround) {
    __shared__ unsigned long long s_lo[SG_MAXLEV][3], s_hi[SG_MAXLEV][3];
    __shared__ unsigned long long s_hmax[SG_MAXLEV], s_cnt[SG_MAXLEV];
    if (g->err & SGE_NONFINITE) return;   // uniform across the grid
    for (int t = threadIdx.x; t < SG_MAXLEV; t += kBlock) {
        for (int d = 0; d < 3; ++d) {
            s_lo[t][d] = ~0ull;
            s_hi[t][d] = 0ull;
        }
        s_hmax[t] = 0ull;
        s_cnt[t] = 0ull;
    }
    __syncthreads();
    const double hmin = sg_unord(g->hmin_bits);
    const double L0 = pow2_ceil(hmin * (2.0 + 0x1p-9));
    bool bad = false;
    for (int64_t r = 0; r < nround; ++r) {
        int64_t i = r * stride + base + threadIdx.x;
        bool valid = i < ng;
        int lev = -1;
        double p[3] = {0, 0, 0}, hi = 0;
        if (valid) {
            hi = h[i];
            p[0] = x[i];
            p[1] = y[i];
            p[2] = z[i];
            lev = level_of(hi, L0);
            if (lev < 0) {
                bad = true;
                valid = false;
            }
        }
        // one LDS atomic per bound and particle: a wavefront's particles
        // arrive in input order and spread over several levels, and seven
        // wavefront reductions per level present had cost more (sort stage
        // at 1M gas 0.427 ms with shuffle reductions, 0.408 with DPP ones,
        // 0.384 with these atomics)
        if (valid) {
            for (int d = 0; d < 3; ++d) {
                atomicMin(&s_lo[lev][d], sg_ord(p[d]));
                atomicMax(&s_hi[lev][d], sg_ord(p[d]));
            }
            atomicMax(&s_hmax[lev], sg_ord(hi));
            atomicAdd(&s_cnt[lev], 1ull);
        }
    }
    if (bad) atomicOr(&g->err, SGE_LEVELS);
    __syncthreads();
    for (int t = threadIdx.x; t < SG_MAXLEV; t += kBlock) {
        if (s_cnt[t] == 0) continue;
        for (int d = 0; d < 3; ++d) {
            atomicMin(&g->lo[t][d], s_lo[t][d]);
            atomicMax(&g->hi[t][d], s_hi[t][d]);
        }
        atomicMax(&g->hmax_bits[t], s_hmax[t]);
        atomicAdd(&g->npart[t], s_cnt[t]);
    }
}

__global__ __launch_bounds__(kBlock) void k_grid_levels(const double* __restrict__ x,
                                                        const double* __restrict__ y,
                                                        const double* __restrict__ z,
                                                        const double* __restrict__ h,
                                                        int64_t ng, sg_grid_dev* g) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    grid_levels_block(x, y, z, h, ng, g, (int64_t)blockIdx.x * kBlock, stride,
                      (ng + stride - 1) / stride);
}

// Cell sides L[l] = L0 2^(l + cell_scale_log2) (powers of two); the level of
// a particle depends on L0 only.
__device__ inline void grid_finish_one(sg_grid_dev* g, int64_t cell_cap, double cell_scale) {
    if (g->err & (SGE_NONFINITE | SGE_LEVELS)) {
        g->M = 0;
        return;
    }
    const double hmin = sg_unord(g->hmin_bits);
    const double L0 = pow2_ceil(hmin * (2.0 + 0x1p-9));
    g->L0 = L0;
    int nlev = 0;
    for (int l = 0; l < SG_MAXLEV; ++l)
        if (g->npart[l]) nlev = l + 1;
    g->nlev = nlev;
    int64_t M = 0;
    double L = L0 * cell_scale;        // exact: cell_scale is 1/2, 1 or 2
    for (int l = 0; l < SG_MAXLEV; ++l, L *= 2.0) {
        g->L[l] = L;
        g->invL[l] = 1.0 / L;          // exact: L is a power of two
        g->base[l] = M;
        g->hmaxlev[l] = g->npart[l] ? sg_unord(g->hmax_bits[l]) : 0.0;
        if (l >= nlev || g->npart[l] == 0) {
            g->ncell[l] = 0;
            for (int d = 0; d < 3; ++d) {
                g->dim[l][d] = 0;
                g->org[l][d] = 0.0;
            }
            continue;
        }
        int64_t nc = 1;
        for (int d = 0; d < 3; ++d) {
            double lo = sg_unord(g->lo[l][d]), hi = sg_unord(g->hi[l][d]);
            double o = floor(lo * g->invL[l]) * L;
            g->org[l][d] = o;
            double span = floor((hi - o) * g->invL[l]);
            if (!(span < 2147483646.0)) {
                atomicOr(&g->err, SGE_GRID);
                g->M = 0;
                return;
            }
            g->dim[l][d] = (int64_t)span + 1;
            nc *= g->dim[l][d];
            if (nc > 2147483647ll) {
                atomicOr(&g->err, SGE_GRID);
                g->M = 0;
                return;
            }
        }
        g->ncell[l] = nc;
        M += nc;
        if (M > 2147483647ll) {
            atomicOr(&g->err, SGE_GRID);
            g->M = 0;
            return;
        }
    }
    g->M = M;
    if (M > cell_cap) {
        atomicOr(&g->err, SGE_CELLS);
        g->need_cells = M;
    }
}

__global__ void k_grid_finish(sg_grid_dev* g, int64_t cell_cap, double cell_scale) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    grid_finish_one(g, cell_cap, cell_scale);
}

__device__ inline void cells_clear_block(const sg_grid_dev* g, int32_t* __restrict__ count,
                                         unsigned long long* __restrict__ hmax, int64_t b,
                                         int64_t nb) {
    if (g->err & SGE_SORT_FATAL) return;
    const int64_t M = g->M;
    for (int64_t k = b * kBlock + threadIdx.x; k < M; k += nb * kBlock) {
        count[k] = 0;
        hmax[k] = 0ull;
    }
}

__global__ __launch_bounds__(kBlock) void k_cells_clear(const sg_grid_dev* g,
                                                        int32_t* __restrict__ count,
                                                        unsigned long long* __restrict__ hmax) {
    cells_clear_block(g, count, hmax, blockIdx.x, gridDim.x);
}

// Cell key of gas particle i, its count and the cell's maximum h.  Every
// lane of the wavefront calls this (valid or not): the lanes that share the
// key of the first valid lane add their count and maximum h with one
// atomic each (clustered or coincident gas puts many particles of a
// wavefront in one cell); the others add their own.
__device__ inline void keys_count_wave(const double* __restrict__ x, const double* __restrict__ y,
                                       const double* __restrict__ z,
                                       const double* __restrict__ h,
                                       const double* __restrict__ m, int64_t i, bool valid,
                                       const sg_grid_dev* g, int32_t* __restrict__ key,
                                       int32_t* __restrict__ count,
                                       unsigned long long* __restrict__ hmax,
                                       sg_prec* __restrict__ pin) {
    int32_t k = -1;
    unsigned long long hb = 0ull;
    if (valid) {
        const double hi = h[i];
        const int l = level_of(hi, g->L0);
        const double p[3] = {x[i], y[i], z[i]};
        // the particle's record in particle order, for the gather
        pin[i] = sg_prec{p[0], p[1], p[2], hi, m[i], {0.0, 0.0, 0.0}};
        int64_t c[3];
        for (int d = 0; d < 3; ++d) {
            double v = floor((p[d] - g->org[l][d]) * g->invL[l]);
            double top = (double)(g->dim[l][d] - 1);
            v = v < 0.0 ? 0.0 : (v > top ? top : v);
            c[d] = (int64_t)v;
        }
        k = (int32_t)(g->base[l] + (c[2] * g->dim[l][1] + c[1]) * g->dim[l][0] + c[0]);
        key[i] = k;
        hb = (unsigned long long)__builtin_bit_cast(long long, hi);   // h > 0: orders as bits
    }
    bool done = !valid;
    const unsigned long long act = __ballot(valid);
    if (act) {
        const int lead = __builtin_ctzll(act);
        const int32_t lk = __builtin_amdgcn_readlane(k, lead);
        const unsigned long long peers = __ballot(valid && k == lk);
        if (__builtin_popcountll(peers) > 1) {
            const bool mine = (peers >> lane_id()) & 1ull;
            const unsigned long long hm = wave_max_u64(mine ? hb : 0ull);
            if ((int)lane_id() == lead) {
                atomicAdd(&count[lk], (int32_t)__builtin_popcountll(peers));
                atomicMax(&hmax[lk], hm);
            }
            done = done || mine;
        }
    }
    if (!done) {
        atomicAdd(&count[k], 1);
        atomicMax(&hmax[k], hb);
    }
}

__global__ __launch_bounds__(kBlock) void k_keys_count(const double* __restrict__ x,
                                                       const double* __restrict__ y,
                                                       const double* __restrict__ z,
                                                       const double* __restrict__ h,
                                                       const double* __restrict__ m,
                                                       int64_t ng, const sg_grid_dev* g,
                                                       int32_t* __restrict__ key,
                                                       int32_t* __restrict__ count,
                                                       unsigned long long* __restrict__ hmax,
                                                       sg_prec* __restrict__ pin) {
    if (g->err & SGE_SORT_FATAL) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    keys_count_wave(x, y, z, h, m, i, i < ng, g, key, count, hmax, pin);
}

// The stable order of the gas by cell key (ascending particle id inside a
// cell) comes from an LSD radix sort of the keys, sg_launch_gas_order;
// here the gather of the sorted state.  The particles arrive in any order,
// so the gather is random: it reads each particle's 64-byte record that
// the key pass wrote in particle order (one aligned line per particle)
// instead of five scattered doubles (five lines): at 1M gas its fetched
// bytes fell from 625 MB to about 130 MB.
__device__ inline void gather_one(const int32_t* __restrict__ perm, int64_t s,
                                  const sg_prec* __restrict__ pin, double* __restrict__ xs,
                                  double* __restrict__ ys, double* __restrict__ zs,
                                  double* __restrict__ hs, double* __restrict__ ms,
                                  sg_prec* __restrict__ prec) {
    const sg_prec r = pin[perm[s]];
    xs[s] = r.x;
    ys[s] = r.y;
    zs[s] = r.z;
    hs[s] = r.h;
    ms[s] = r.m;
    prec[s] = r;
}

__global__ __launch_bounds__(kBlock) void k_gather_gas(
    const int32_t* __restrict__ perm, int64_t ng, const sg_grid_dev* g,
    const sg_prec* __restrict__ pin, double* __restrict__ xs, double* __restrict__ ys,
    double* __restrict__ zs, double* __restrict__ hs, double* __restrict__ ms,
    sg_prec* __restrict__ prec) {
    if (g->err & SGE_SORT_FATAL) return;
    int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= ng) return;
    gather_one(perm, s, pin, xs, ys, zs, hs, ms, prec);
}

// ------------------------------------------------------ Morton ordering --

constexpr int kRadixItems = 16;
constexpr int kRadixTile = kBlock * kRadixItems;

__global__ void k_gbox_reset(sg_grid_dev* g) {
    if (threadIdx.x < 3) {
        g->glo[threadIdx.x] = ~0ull;
        g->ghi[threadIdx.x] = 0ull;
    }
}

// Fold one thread's bounds into the grid record: wavefront, then
// workgroup, then one global atomic per bound and workgroup (same-address
// atomics from every wavefront serialise in L2).
__device__ inline void gbox_fold(const unsigned long long (&mn)[3], const unsigned long long (&mx)[3],
                                 bool bad, sg_grid_dev* g) {
    __shared__ unsigned long long s_lo[3][kBlock / 64], s_hi[3][kBlock / 64];
    const int w = threadIdx.x >> 6;
    for (int d = 0; d < 3; ++d) {
        unsigned long long a = wave_min_u64(mn[d]), b = wave_max_u64(mx[d]);
        if (lane_id() == 0) {
            s_lo[d][w] = a;
            s_hi[d][w] = b;
        }
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int d = threadIdx.x;
        unsigned long long a = s_lo[d][0], b = s_hi[d][0];
        for (int k = 1; k < kBlock / 64; ++k) {
            a = s_lo[d][k] < a ? s_lo[d][k] : a;
            b = s_hi[d][k] > b ? s_hi[d][k] : b;
        }
        atomicMin(&g->glo[d], a);
        atomicMax(&g->ghi[d], b);
    }
    if (bad) atomicOr(&g->err, SGE_GNONFINITE);
}

__device__ inline void gbox_point(const double* __restrict__ x, const double* __restrict__ y,
                                  const double* __restrict__ z, int64_t i,
                                  unsigned long long (&mn)[3], unsigned long long (&mx)[3],
                                  bool& bad) {
    const double p[3] = {x[i], y[i], z[i]};
    for (int d = 0; d < 3; ++d) {
        if (!finite_d(p[d])) {
            bad = true;
            continue;
        }
        unsigned long long o = sg_ord(p[d]);
        mn[d] = o < mn[d] ? o : mn[d];
        mx[d] = o > mx[d] ? o : mx[d];
    }
}

__global__ __launch_bounds__(kBlock) void k_gbox(const double* __restrict__ x,
                                                 const double* __restrict__ y,
                                                 const double* __restrict__ z, int64_t n,
                                                 sg_grid_dev* g) {
    unsigned long long mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {0, 0, 0};
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        gbox_point(x, y, z, i, mn, mx, bad);
    gbox_fold(mn, mx, bad, g);
}

__device__ inline uint32_t spread3(uint32_t v) {   // 10 bits -> every third bit
    v &= 0x3ff;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ inline void morton_key_one(const double* __restrict__ x, const double* __restrict__ y,
                                      const double* __restrict__ z, int64_t i,
                                      const sg_grid_dev* g, uint32_t* __restrict__ keys,
                                      int32_t* __restrict__ vals) {
    double lo[3], ext = 0.0;
    for (int d = 0; d < 3; ++d) {
        lo[d] = sg_unord(g->glo[d]);
        double e = sg_unord(g->ghi[d]) - lo[d];
        ext = e > ext ? e : ext;
    }
    const double scale = ext > 0.0 ? 1024.0 / (ext * (1.0 + 0x1p-20)) : 0.0;
    const double p[3] = {x[i], y[i], z[i]};
    uint32_t c[3];
    for (int d = 0; d < 3; ++d) {
        double v = (p[d] - lo[d]) * scale;
        v = v < 0.0 ? 0.0 : (v > 1023.0 ? 1023.0 : v);
        c[d] = (uint32_t)v;
    }
    keys[i] = spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2);
    vals[i] = (int32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_morton_keys(const double* __restrict__ x,
                                                        const double* __restrict__ y,
                                                        const double* __restrict__ z, int64_t n,
                                                        const sg_grid_dev* g,
                                                        uint32_t* __restrict__ keys,
                                                        int32_t* __restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    morton_key_one(x, y, z, i, g, keys, vals);
}

// Morton keys have 30 bits: three passes of 10-bit digits.
constexpr int kRadixBits = 10;
constexpr int kBuckets = 1 << kRadixBits;
constexpr int kRadixPasses = 3;

// Digit histogram of one tile, stored digit-major: hist[d * ntiles + tile].
__device__ inline void radix_hist_tile(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                       int64_t ntiles, int32_t* __restrict__ hist,
                                       int64_t tile) {
    __shared__ int32_t s_h[kBuckets];
    for (int t = threadIdx.x; t < kBuckets; t += kBlock) s_h[t] = 0;
    __syncthreads();
    const int64_t base = tile * kRadixTile;
    for (int k = 0; k < kRadixItems; ++k) {
        int64_t i = base + k * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&s_h[(keys[i] >> shift) & (kBuckets - 1)], 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kBuckets; t += kBlock) hist[(int64_t)t * ntiles + tile] = s_h[t];
}

__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                       int64_t n, int shift, int64_t ntiles,
                                                       int32_t* __restrict__ hist) {
    radix_hist_tile(keys, n, shift, ntiles, hist, blockIdx.x);
}

// Stable scatter: element order inside the tile is preserved within each
// digit (chunk by chunk, wave by wave, lane by lane).  Per chunk, the first
// lane of each (wave, digit) group publishes the group's size; after the
// writes it adds that size to the digit's running count and clears its slot.
// vin == nullptr stands for the values 0, 1, 2, .. (the element indices).
__device__ inline void radix_scatter_tile(const uint32_t* __restrict__ kin,
                                          const int32_t* __restrict__ vin, int64_t n, int shift,
                                          int64_t ntiles, const int64_t* __restrict__ offs,
                                          uint32_t* __restrict__ kout,
                                          int32_t* __restrict__ vout, int64_t tile) {
    // a (wave, digit) group of one chunk has at most 64 members: one byte
    // each keeps the workgroup's LDS at 8 KB, small enough to find room on
    // CUs that a persistent gravity kernel mostly fills
    __shared__ int32_t s_run[kBuckets];
    __shared__ uint8_t s_w[kBlock / 64][kBuckets];
    const int wave = threadIdx.x >> 6;
    for (int t = threadIdx.x; t < kBuckets; t += kBlock) {
        s_run[t] = 0;
        for (int w = 0; w < kBlock / 64; ++w) s_w[w][t] = 0;
    }
    __syncthreads();
    const int64_t base = tile * kRadixTile;
    for (int k = 0; k < kRadixItems; ++k) {
        const int64_t i = base + k * kBlock + threadIdx.x;
        const bool valid = i < n;
        const uint32_t key = valid ? kin[i] : 0u;
        const int32_t val = valid ? (vin ? vin[i] : (int32_t)i) : 0;
        const uint32_t d = (key >> shift) & (kBuckets - 1);
        unsigned long long peers = __ballot(valid);
        for (int b = 0; b < kRadixBits; ++b) {
            unsigned long long bb = __ballot(valid && ((d >> b) & 1u));
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        const unsigned r = rank_below(peers);
        const int cnt = __builtin_popcountll(peers);
        const bool lead = valid && r == 0;
        if (lead) s_w[wave][d] = (uint8_t)cnt;
        __syncthreads();
        if (valid) {
            int32_t pre = 0;
            for (int w = 0; w < wave; ++w) pre += s_w[w][d];
            const int64_t dest = offs[(int64_t)d * ntiles + tile] + s_run[d] + pre + r;
            kout[dest] = key;
            vout[dest] = val;
        }
        __syncthreads();
        if (lead) {
            atomicAdd(&s_run[d], cnt);
            s_w[wave][d] = 0;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin, int64_t n, int shift,
    int64_t ntiles, const int64_t* __restrict__ offs, uint32_t* __restrict__ kout,
    int32_t* __restrict__ vout) {
    radix_scatter_tile(kin, vin, n, shift, ntiles, offs, kout, vout, blockIdx.x);
}

// ---------------------------------------- Morton order, all systems at once --
// (see sg_seg in sg_internal.h).  The same stable order as the per-system
// sort: the same keys, digits and stable scatter.

__global__ void k_seg_gbox_reset(const sg_seg_sys* __restrict__ sys, int nsys) {
    for (int k = threadIdx.x; k < nsys; k += blockDim.x) {
        sg_grid_dev* g = sys[k].g;
        for (int d = 0; d < 3; ++d) {
            g->glo[d] = ~0ull;
            g->ghi[d] = 0ull;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_seg_gbox(const sg_seg_sys* __restrict__ sys,
                                                     const int64_t* __restrict__ pfx, int nsys) {
    int64_t lb;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &lb)];
    unsigned long long mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {0, 0, 0};
    bool bad = false;
    const int64_t i = lb * kBlock + threadIdx.x;
    if (i < S.n) gbox_point(S.x, S.y, S.z, i, mn, mx, bad);
    gbox_fold(mn, mx, bad, S.g);
}

__global__ __launch_bounds__(kBlock) void k_seg_morton_keys(const sg_seg_sys* __restrict__ sys,
                                                            const int64_t* __restrict__ pfx,
                                                            int nsys) {
    int64_t lb;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &lb)];
    const int64_t i = lb * kBlock + threadIdx.x;
    if (i < S.n) morton_key_one(S.x, S.y, S.z, i, S.g, S.mk0, S.mv0);
}

// pass p reads buffer p & 1 and writes the other one; the last pass writes
// the values to the order
__global__ __launch_bounds__(kBlock) void k_seg_radix_hist(const sg_seg_sys* __restrict__ sys,
                                                           const int64_t* __restrict__ pfx,
                                                           int nsys, int pass) {
    int64_t tile;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &tile)];
    radix_hist_tile((pass & 1) ? S.mk1 : S.mk0, S.n, kRadixBits * pass, S.ntiles, S.mhist, tile);
}

__global__ __launch_bounds__(kBlock) void k_seg_radix_scatter(const sg_seg_sys* __restrict__ sys,
                                                              const int64_t* __restrict__ pfx,
                                                              int nsys, int pass) {
    int64_t tile;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &tile)];
    const bool odd = pass & 1;
    int32_t* vout = pass == kRadixPasses - 1 ? S.order : (odd ? S.mv0 : S.mv1);
    radix_scatter_tile(odd ? S.mk1 : S.mk0, odd ? S.mv1 : S.mv0, S.n, kRadixBits * pass,
                       S.ntiles, S.moffs, odd ? S.mk0 : S.mk1, vout, tile);
}

// Exclusive scan of one system's digit histogram (1024 * ntiles counts)
// into its offsets, one workgroup per system; offs[total] is not needed by
// the scatter and not written.  gas: the cell-key sort's histogram, else the
// Morton sort's.  256 lanes: the cell-key sort runs beside the persistent
// gravity kernel, and a 1024-lane workgroup (4 free wave slots on every
// SIMD of one CU) waited there for the gravity kernel to end (173 ms).
constexpr int kSegScanBlock = 256;
__global__ __launch_bounds__(kSegScanBlock) void k_seg_scan_hist(const sg_seg_sys* __restrict__ sys,
                                                                 int gas) {
    const sg_seg_sys& S = sys[blockIdx.x];
    const int32_t* hist = gas ? S.ghist : S.mhist;
    int64_t* offs = gas ? S.goffs : S.moffs;
    const int64_t n = (int64_t)kBuckets * (gas ? S.gntiles : S.ntiles);
    __shared__ int64_t s_w[kSegScanBlock / 64];
    __shared__ int64_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    constexpr int kItems = 4;
    for (int64_t c0 = 0; c0 < n; c0 += (int64_t)kSegScanBlock * kItems) {
        const int64_t i0 = c0 + (int64_t)threadIdx.x * kItems;
        int64_t v[kItems], tsum = 0;
        for (int k = 0; k < kItems; ++k) {
            v[k] = i0 + k < n ? hist[i0 + k] : 0;
            tsum += v[k];
        }
        int64_t incl = tsum;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t t = __shfl_up(incl, o, 64);
            if (lane_id() >= (unsigned)o) incl += t;
        }
        if (lane_id() == 63) s_w[threadIdx.x >> 6] = incl;
        __syncthreads();
        int64_t wbase = s_carry;
        for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) wbase += s_w[w];
        int64_t run = wbase + incl - tsum;
        for (int k = 0; k < kItems; ++k) {
            if (i0 + k < n) offs[i0 + k] = run;
            run += v[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t t = 0;
            for (int w = 0; w < kSegScanBlock / 64; ++w) t += s_w[w];
            s_carry += t;
        }
        __syncthreads();
    }
}

// ----------------------------------------- gas sort, all systems at once --
// (see sg_seg in sg_internal.h): the per-system kernels' bodies; a system
// without gas is skipped, as the per-system build does.

__global__ void k_seg_grid_reset(const sg_seg_sys* __restrict__ sys) {
    const sg_seg_sys& S = sys[blockIdx.x];
    if (S.ng > 0) grid_reset_one(S.g);
}

__global__ __launch_bounds__(kBlock) void k_seg_grid_hmin(const sg_seg_sys* __restrict__ sys,
                                                          const int64_t* __restrict__ pfx,
                                                          int nsys) {
    int64_t lb;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &lb)];
    unsigned long long mn = ~0ull;
    bool bad = false;
    const int64_t i = lb * kBlock + threadIdx.x;
    if (i < S.ng) hmin_item(S.x, S.y, S.z, S.h, i, mn, bad);
    hmin_fold(mn, bad, S.g);
}

__global__ __launch_bounds__(kBlock) void k_seg_grid_levels(const sg_seg_sys* __restrict__ sys,
                                                            const int64_t* __restrict__ pfx,
                                                            int nsys) {
    int64_t lb;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &lb)];
    grid_levels_block(S.x, S.y, S.z, S.h, S.ng, S.g, lb * kBlock, 0, 1);
}

__global__ void k_seg_grid_finish(const sg_seg_sys* __restrict__ sys, int nsys) {
    for (int k = threadIdx.x; k < nsys; k += blockDim.x)
        if (sys[k].ng > 0) grid_finish_one(sys[k].g, sys[k].cell_cap, sys[k].cell_scale);
}

__global__ __launch_bounds__(kBlock) void k_seg_cells_clear(const sg_seg_sys* __restrict__ sys,
                                                            const int64_t* __restrict__ pfx,
                                                            int nsys) {
    int64_t lb;
    const int k = sg_seg_find(pfx, nsys, blockIdx.x, &lb);
    const sg_seg_sys& S = sys[k];
    cells_clear_block(S.g, S.count, S.hmax, lb, pfx[k + 1] - pfx[k]);
}

__global__ __launch_bounds__(kBlock) void k_seg_keys_count(const sg_seg_sys* __restrict__ sys,
                                                           const int64_t* __restrict__ pfx,
                                                           int nsys) {
    int64_t lb;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &lb)];
    if (S.g->err & SGE_SORT_FATAL) return;
    const int64_t i = lb * kBlock + threadIdx.x;
    keys_count_wave(S.x, S.y, S.z, S.h, S.m, i, i < S.ng, S.g, S.key, S.count, S.hmax,
                    reinterpret_cast<sg_prec*>(S.sph.f64));
}

// which = 0: cell counts -> cell offsets (n = M from the grid, bounded by
// the cell capacity); 1: neighbour counts -> CSR offsets (n = N_g)
__device__ inline void seg_scan_args(const sg_seg_sys& S, int which, const int32_t** in,
                                     int64_t** out, int64_t* n) {
    if (which == 0) {
        *in = S.count;
        *out = S.off;
        *n = S.g->M < S.cell_cap ? S.g->M : S.cell_cap;
    } else {
        *in = S.ncnt;
        *out = const_cast<int64_t*>(S.sph.nbr_off);
        *n = S.ng;
    }
}

__global__ __launch_bounds__(kBlock) void k_seg_scan_reduce(const sg_seg_sys* __restrict__ sys,
                                                            const int64_t* __restrict__ pfx,
                                                            int nsys, int which) {
    int64_t tile;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &tile)];
    const int32_t* in;
    int64_t* out;
    int64_t n;
    seg_scan_args(S, which, &in, &out, &n);
    scan_reduce_tile(in, n, tile, (int64_t*)S.scan);
}

__global__ __launch_bounds__(256) void k_seg_scan_bsums(const sg_seg_sys* __restrict__ sys,
                                                        int which) {
    const sg_seg_sys& S = sys[blockIdx.x];
    if (S.ng == 0) return;
    const int32_t* in;
    int64_t* out;
    int64_t n;
    seg_scan_args(S, which, &in, &out, &n);
    scan_bsums_block((int64_t*)S.scan, n, out);
}

__global__ __launch_bounds__(kBlock) void k_seg_scan_down(const sg_seg_sys* __restrict__ sys,
                                                          const int64_t* __restrict__ pfx,
                                                          int nsys, int which) {
    int64_t tile;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &tile)];
    const int32_t* in;
    int64_t* out;
    int64_t n;
    seg_scan_args(S, which, &in, &out, &n);
    scan_down_tile(in, out, n, tile, (const int64_t*)S.scan);
}

// Cell-key radix pass `pass` of every system (the per-system buffers'
// ping-pong of sg_launch_gas_order); the last pass writes the order.
__device__ inline void seg_gas_bufs(const sg_seg_sys& S, int pass, const uint32_t** kin,
                                    const int32_t** vin) {
    *kin = pass == 0 ? (const uint32_t*)S.key : (((pass - 1) & 1) ? S.gk1 : S.gk0);
    *vin = pass == 0 ? nullptr : (((pass - 1) & 1) ? S.gv1 : S.gv0);
}

__global__ __launch_bounds__(kBlock) void k_seg_gas_hist(const sg_seg_sys* __restrict__ sys,
                                                         const int64_t* __restrict__ pfx,
                                                         int nsys, int pass) {
    int64_t tile;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &tile)];
    const uint32_t* kin;
    const int32_t* vin;
    seg_gas_bufs(S, pass, &kin, &vin);
    radix_hist_tile(kin, S.ng, kRadixBits * pass, S.gntiles, S.ghist, tile);
}

__global__ __launch_bounds__(kBlock) void k_seg_gas_scatter(const sg_seg_sys* __restrict__ sys,
                                                            const int64_t* __restrict__ pfx,
                                                            int nsys, int pass, int last) {
    int64_t tile;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &tile)];
    const uint32_t* kin;
    const int32_t* vin;
    seg_gas_bufs(S, pass, &kin, &vin);
    int32_t* vout = last ? const_cast<int32_t*>(S.sph.perm) : ((pass & 1) ? S.gv1 : S.gv0);
    radix_scatter_tile(kin, vin, S.ng, kRadixBits * pass, S.gntiles, S.goffs,
                       (pass & 1) ? S.gk1 : S.gk0, vout, tile);
}

__global__ __launch_bounds__(kBlock) void k_seg_gather_gas(const sg_seg_sys* __restrict__ sys,
                                                           const int64_t* __restrict__ pfx,
                                                           int nsys) {
    int64_t lb;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &lb)];
    if (S.g->err & SGE_SORT_FATAL) return;
    const int64_t s = lb * kBlock + threadIdx.x;
    const sg_sph_bufs& b = S.sph;
    if (s < S.ng)
        gather_one(b.perm, s, reinterpret_cast<const sg_prec*>(b.f64), b.xs, b.ys, b.zs, b.hs,
                   b.ms, b.prec);
}

inline unsigned grid_for(int64_t n, int per_block) {
    int64_t b = (n + per_block - 1) / per_block;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

// ----------------------------------------------------------- launchers --

size_t sg_scan_tmp_bytes(int64_t cap) {
    return sizeof(int64_t) * (size_t)((cap + kScanTile - 1) / kScanTile + 1);
}

void sg_launch_scan(const int32_t* in, int64_t* out, int64_t n_host, const int64_t* n_dev,
                    int64_t cap, void* tmp, hipStream_t st) {
    const unsigned nb = grid_for(cap, kScanTile);
    int64_t* bsum = (int64_t*)tmp;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, st, in, n_host, n_dev, cap, bsum);
    hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(256), 0, st, bsum, n_host, n_dev, cap, out);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kBlock), 0, st, in, out, n_host, n_dev, cap,
                       bsum);
}

void sg_launch_grid_reset(sg_grid_dev* g, hipStream_t st) {
    hipLaunchKernelGGL(k_grid_reset, dim3(1), dim3(64), 0, st, g);
}

void sg_launch_status_clear(sg_grid_dev* g, hipStream_t st) {
    hipLaunchKernelGGL(k_status_clear, dim3(1), dim3(64), 0, st, g);
}

void sg_launch_grid_reduce(const double* x, const double* y, const double* z, const double* h,
                           int64_t ng, sg_grid_dev* g, hipStream_t st) {
    unsigned nb = grid_for(ng, kBlock);
    if (nb > 1024) nb = 1024;
    hipLaunchKernelGGL(k_grid_hmin, dim3(nb), dim3(kBlock), 0, st, x, y, z, h, ng, g);
    hipLaunchKernelGGL(k_grid_levels, dim3(nb), dim3(kBlock), 0, st, x, y, z, h, ng, g);
}

void sg_launch_grid_finish(sg_grid_dev* g, int64_t cell_cap, int cell_scale_log2, hipStream_t st) {
    const double scale = cell_scale_log2 < 0 ? 0.5 : (cell_scale_log2 > 0 ? 2.0 : 1.0);
    hipLaunchKernelGGL(k_grid_finish, dim3(1), dim3(64), 0, st, g, cell_cap, scale);
}

void sg_launch_cells_clear(sg_grid_dev* g, int32_t* count, unsigned long long* hmax,
                           int64_t cell_cap, hipStream_t st) {
    unsigned nb = grid_for(cell_cap, kBlock);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_cells_clear, dim3(nb), dim3(kBlock), 0, st, g, count, hmax);
}

void sg_launch_keys_count(const double* x, const double* y, const double* z, const double* h,
                          const double* m, int64_t ng, sg_grid_dev* g, int32_t* key,
                          int32_t* count, unsigned long long* hmax, sg_prec* pin,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_keys_count, dim3(grid_for(ng, kBlock)), dim3(kBlock), 0, st, x, y, z,
                       h, m, ng, g, key, count, hmax, pin);
}

void sg_launch_gather_gas(const int32_t* perm, int64_t ng, const sg_grid_dev* g,
                          const sg_prec* pin, double* xs, double* ys, double* zs, double* hs,
                          double* ms, sg_prec* prec, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_gas, dim3(grid_for(ng, kBlock)), dim3(kBlock), 0, st, perm, ng,
                       g, pin, xs, ys, zs, hs, ms, prec);
}

// Workspace of the Morton order: two key/value buffers, the digit histogram
// and its offsets, and the scan scratch.
static void morton_layout(int64_t n, size_t* o_k1, size_t* o_v0, size_t* o_v1, size_t* o_hist,
                          size_t* o_offs, size_t* o_scan, size_t* total) {
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
    const int64_t nh = kBuckets * (ntiles > 0 ? ntiles : 1);
    size_t o = 0;
    o += al(sizeof(uint32_t) * (size_t)n);  // k0 at 0
    *o_k1 = o;
    o += al(sizeof(uint32_t) * (size_t)n);
    *o_v0 = o;
    o += al(sizeof(int32_t) * (size_t)n);
    *o_v1 = o;
    o += al(sizeof(int32_t) * (size_t)n);
    *o_hist = o;
    o += al(sizeof(int32_t) * (size_t)nh);
    *o_offs = o;
    o += al(sizeof(int64_t) * (size_t)(nh + 1));
    *o_scan = o;
    o += al(sg_scan_tmp_bytes(nh));
    *total = o;
}

size_t sg_morton_tmp_bytes(int64_t n) {
    size_t a, b, c, d, e, f, t;
    morton_layout(n, &a, &b, &c, &d, &e, &f, &t);
    return t;
}

int64_t sg_radix_tiles(int64_t n) { return (n + kRadixTile - 1) / kRadixTile; }
int64_t sg_scan_tiles(int64_t cap) { return grid_for(cap, kScanTile); }
int64_t sg_cells_clear_blocks(int64_t cell_cap) {
    const int64_t nb = grid_for(cell_cap, kBlock);
    return nb > 256 ? 256 : nb;
}

static void seg_scan(const sg_seg& s, int which, hipStream_t st) {
    const int q = which == 0 ? SG_SEG_SCAN_C : SG_SEG_SCAN_G;
    const int64_t* p = s.pfx + q * (s.nsys + 1);
    if (s.nblk[q] == 0) return;
    hipLaunchKernelGGL(k_seg_scan_reduce, dim3((unsigned)s.nblk[q]), dim3(kBlock), 0, st, s.sys, p,
                       s.nsys, which);
    hipLaunchKernelGGL(k_seg_scan_bsums, dim3((unsigned)s.nsys), dim3(256), 0, st, s.sys, which);
    hipLaunchKernelGGL(k_seg_scan_down, dim3((unsigned)s.nblk[q]), dim3(kBlock), 0, st, s.sys, p,
                       s.nsys, which);
}

void sg_seg_launch_sort(const sg_seg& s, hipStream_t st) {
    if (s.nblk[SG_SEG_NG] == 0) return;
    const int64_t* png = s.pfx + SG_SEG_NG * (s.nsys + 1);
    const int64_t* pcl = s.pfx + SG_SEG_CELLS * (s.nsys + 1);
    const unsigned nbg = (unsigned)s.nblk[SG_SEG_NG];
    hipLaunchKernelGGL(k_seg_grid_reset, dim3((unsigned)s.nsys), dim3(64), 0, st, s.sys);
    hipLaunchKernelGGL(k_seg_grid_hmin, dim3(nbg), dim3(kBlock), 0, st, s.sys, png, s.nsys);
    hipLaunchKernelGGL(k_seg_grid_levels, dim3(nbg), dim3(kBlock), 0, st, s.sys, png, s.nsys);
    hipLaunchKernelGGL(k_seg_grid_finish, dim3(1), dim3(64), 0, st, s.sys, s.nsys);
    hipLaunchKernelGGL(k_seg_cells_clear, dim3((unsigned)s.nblk[SG_SEG_CELLS]), dim3(kBlock), 0, st,
                       s.sys, pcl, s.nsys);
    hipLaunchKernelGGL(k_seg_keys_count, dim3(nbg), dim3(kBlock), 0, st, s.sys, png, s.nsys);
    seg_scan(s, 0, st);
    const int64_t* pgt = s.pfx + SG_SEG_GTILES * (s.nsys + 1);
    for (int pass = 0; pass < s.gas_passes; ++pass) {
        hipLaunchKernelGGL(k_seg_gas_hist, dim3((unsigned)s.nblk[SG_SEG_GTILES]), dim3(kBlock), 0,
                           st, s.sys, pgt, s.nsys, pass);
        hipLaunchKernelGGL(k_seg_scan_hist, dim3((unsigned)s.nsys), dim3(kSegScanBlock), 0, st,
                           s.sys, 1);
        hipLaunchKernelGGL(k_seg_gas_scatter, dim3((unsigned)s.nblk[SG_SEG_GTILES]), dim3(kBlock),
                           0, st, s.sys, pgt, s.nsys, pass, pass == s.gas_passes - 1 ? 1 : 0);
    }
    hipLaunchKernelGGL(k_seg_gather_gas, dim3(nbg), dim3(kBlock), 0, st, s.sys, png, s.nsys);
}

void sg_seg_launch_scan_nbr(const sg_seg& s, hipStream_t st) { seg_scan(s, 1, st); }

void sg_morton_ptrs(void* tmp, int64_t n, uint32_t** k0, uint32_t** k1, int32_t** v0,
                    int32_t** v1, int32_t** hist, int64_t** offs, int64_t* ntiles) {
    size_t o_k1, o_v0, o_v1, o_hist, o_offs, o_scan, total;
    morton_layout(n, &o_k1, &o_v0, &o_v1, &o_hist, &o_offs, &o_scan, &total);
    char* base = (char*)tmp;
    *k0 = (uint32_t*)base;
    *k1 = (uint32_t*)(base + o_k1);
    *v0 = (int32_t*)(base + o_v0);
    *v1 = (int32_t*)(base + o_v1);
    *hist = (int32_t*)(base + o_hist);
    *offs = (int64_t*)(base + o_offs);
    *ntiles = sg_radix_tiles(n);
}

void sg_seg_launch_morton_order(const sg_seg& s, hipStream_t st) {
    const int64_t* pn = s.pfx + SG_SEG_N * (s.nsys + 1);
    const int64_t* pt = s.pfx + SG_SEG_TILES * (s.nsys + 1);
    if (s.nblk[SG_SEG_N] == 0) return;
    hipLaunchKernelGGL(k_seg_gbox_reset, dim3(1), dim3(64), 0, st, s.sys, s.nsys);
    hipLaunchKernelGGL(k_seg_gbox, dim3((unsigned)s.nblk[SG_SEG_N]), dim3(kBlock), 0, st, s.sys, pn,
                       s.nsys);
    hipLaunchKernelGGL(k_seg_morton_keys, dim3((unsigned)s.nblk[SG_SEG_N]), dim3(kBlock), 0, st,
                       s.sys, pn, s.nsys);
    for (int pass = 0; pass < kRadixPasses; ++pass) {
        hipLaunchKernelGGL(k_seg_radix_hist, dim3((unsigned)s.nblk[SG_SEG_TILES]), dim3(kBlock), 0,
                           st, s.sys, pt, s.nsys, pass);
        hipLaunchKernelGGL(k_seg_scan_hist, dim3((unsigned)s.nsys), dim3(kSegScanBlock), 0, st,
                           s.sys, 0);
        hipLaunchKernelGGL(k_seg_radix_scatter, dim3((unsigned)s.nblk[SG_SEG_TILES]), dim3(kBlock),
                           0, st, s.sys, pt, s.nsys, pass);
    }
}

int sg_gas_radix_passes(int64_t cell_cap) {
    uint64_t top = cell_cap > 1 ? (uint64_t)(cell_cap - 1) : 1u;   // largest key
    int bits = 0;
    while (top) {
        ++bits;
        top >>= 1;
    }
    return (bits + kRadixBits - 1) / kRadixBits;
}

void sg_launch_gas_order(const int32_t* key, int64_t ng, int64_t cell_cap, void* tmp,
                         int32_t* perm, hipStream_t st) {
    uint32_t *k0, *k1;
    int32_t *v0, *v1, *hist;
    int64_t* offs;
    int64_t ntiles;
    sg_morton_ptrs(tmp, ng, &k0, &k1, &v0, &v1, &hist, &offs, &ntiles);
    size_t o_k1, o_v0, o_v1, o_hist, o_offs, o_scan, total;
    morton_layout(ng, &o_k1, &o_v0, &o_v1, &o_hist, &o_offs, &o_scan, &total);
    void* scan_tmp = (char*)tmp + o_scan;
    uint32_t* kb[2] = {k0, k1};
    int32_t* vb[2] = {v0, v1};
    const int passes = sg_gas_radix_passes(cell_cap);
    const uint32_t* kin = (const uint32_t*)key;        // keys are >= 0
    const int32_t* vin = nullptr;                        // ids 0 .. ng-1
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = kRadixBits * pass;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)ntiles), dim3(kBlock), 0, st, kin, ng,
                           shift, ntiles, hist);
        sg_launch_scan(hist, offs, kBuckets * ntiles, nullptr, kBuckets * ntiles, scan_tmp, st);
        int32_t* vout = pass == passes - 1 ? perm : vb[pass & 1];
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)ntiles), dim3(kBlock), 0, st, kin, vin,
                           ng, shift, ntiles, offs, kb[pass & 1], vout);
        kin = kb[pass & 1];
        vin = vb[pass & 1];
    }
}

void sg_launch_morton_order(const double* x, const double* y, const double* z, int64_t n,
                            sg_grid_dev* g, int32_t* order, void* tmp, hipStream_t st) {
    size_t o_k1, o_v0, o_v1, o_hist, o_offs, o_scan, total;
    morton_layout(n, &o_k1, &o_v0, &o_v1, &o_hist, &o_offs, &o_scan, &total);
    char* base = (char*)tmp;
    uint32_t* k[2] = {(uint32_t*)base, (uint32_t*)(base + o_k1)};
    int32_t* v[2] = {(int32_t*)(base + o_v0), (int32_t*)(base + o_v1)};
    int32_t* hist = (int32_t*)(base + o_hist);
    int64_t* offs = (int64_t*)(base + o_offs);
    void* scan_tmp = base + o_scan;
    const int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
    unsigned nb = grid_for(n, kBlock);
    hipLaunchKernelGGL(k_gbox_reset, dim3(1), dim3(64), 0, st, g);
    hipLaunchKernelGGL(k_gbox, dim3(nb > 512 ? 512 : nb), dim3(kBlock), 0, st, x, y, z, n, g);
    hipLaunchKernelGGL(k_morton_keys, dim3(nb), dim3(kBlock), 0, st, x, y, z, n, g, k[0], v[0]);
    int cur = 0;
    for (int pass = 0; pass < kRadixPasses; ++pass) {
        const int shift = kRadixBits * pass;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)ntiles), dim3(kBlock), 0, st, k[cur], n,
                           shift, ntiles, hist);
        sg_launch_scan(hist, offs, kBuckets * ntiles, nullptr, kBuckets * ntiles, scan_tmp, st);
        int32_t* vo = (pass == kRadixPasses - 1) ? order : v[cur ^ 1];
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)ntiles), dim3(kBlock), 0, st, k[cur],
                           v[cur], n, shift, ntiles, offs, k[cur ^ 1], vo);
        cur ^= 1;
    }
}

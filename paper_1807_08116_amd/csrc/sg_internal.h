// sg_internal.h -- device-side structures and launcher declarations shared by
// the translation units of libsphgrav.so (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sphgrav.h"

#define SG_MAXLEV SG_MAX_LEVELS

// Device error bits (latched; cleared by sg_create / sg_bind_state).
enum : uint32_t {
    SGE_LEVELS = 1u,      // smoothing lengths need more than SG_MAXLEV levels
    SGE_CELLS = 2u,       // M > cell_cap
    SGE_NNZ = 4u,         // neighbour pairs > nnz_cap
    SGE_NONFINITE = 8u,   // non-finite position, h <= 0 or non-finite h
    SGE_GRID = 16u,       // a level's cell count does not fit in int32
    SGE_GNONFINITE = 32u, // non-finite position met by the gravity preparation
                          // (apart from SGE_NONFINITE, which the neighbour
                          // build reads: the two chains may run concurrently)
};
#define SGE_SORT_FATAL (SGE_LEVELS | SGE_CELLS | SGE_NONFINITE | SGE_GRID)

// Grid of smoothing-length levels plus the device status word.  Lives in
// the workspace; written only by device code: the level fields by the
// neighbour build, the gravity-order box (glo, ghi) by the gravity
// preparation, the status word by both (atomic OR).
// Workgroups of a launch are dealt to the 8 XCDs of the chip round-robin,
// and each XCD has its own L2.  Kernels whose neighbouring targets share
// data (neighbour gathers over slot-ordered particles) remap the block
// index so that each XCD walks one contiguous range of blocks: a bijection
// of [0, nb), whatever the hardware's actual placement.
constexpr int kXcds = 8;
__device__ inline int64_t xcd_block(int64_t b, int64_t nb) {
    const int64_t per = nb / kXcds, rem = nb % kXcds;
    const int64_t x = b % kXcds, k = b / kXcds;
    return x * per + (x < rem ? x : rem) + k;
}

// Chunked variant: chunks of G consecutive logical blocks are dealt to the
// XCDs in turn, so every XCD takes work from all parts of the range while
// the blocks of one chunk share an L2.  Blocks in the tail (the last
// nb mod 8G) keep their own index.  A bijection of [0, nb).
__device__ inline int64_t xcd_chunk_block(int64_t b, int64_t nb, int64_t G) {
    const int64_t span = kXcds * G;
    if (b >= nb / span * span) return b;
    const int64_t x = b % kXcds, k = b / kXcds;
    return ((k / G) * kXcds + x) * G + k % G;
}

// System of block b of a segmented launch: the largest s with p[s] <= b
// (p = per-system prefix of block counts, p[0] = 0; systems without blocks
// are never found); *local = b - p[s].
__device__ inline int sg_seg_find(const int64_t* __restrict__ p, int nsys, int64_t b,
                                  int64_t* local) {
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (p[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    *local = b - p[lo];
    return lo;
}

struct sg_grid_dev {
    // reduction inputs (order-preserving u64 images of doubles)
    unsigned long long hmin_bits;
    unsigned long long lo[SG_MAXLEV][3];
    unsigned long long hi[SG_MAXLEV][3];
    unsigned long long hmax_bits[SG_MAXLEV];
    unsigned long long npart[SG_MAXLEV];
    // finished grid
    double L0;
    double L[SG_MAXLEV], invL[SG_MAXLEV];
    double org[SG_MAXLEV][3];
    int64_t dim[SG_MAXLEV][3];
    int64_t base[SG_MAXLEV];
    int64_t ncell[SG_MAXLEV];
    double hmaxlev[SG_MAXLEV];
    int32_t nlev, pad0;
    int64_t M;
    // gravity-order bounding box over all N (order-preserving u64 images)
    unsigned long long glo[3], ghi[3];
    // status
    uint32_t err, pad1;
    int64_t need_cells, need_nnz;
    int64_t nnz;
};

// Order-preserving map of doubles onto u64 (for integer atomic min/max).
__host__ __device__ inline unsigned long long sg_ord(double v) {
    unsigned long long b = (unsigned long long)__builtin_bit_cast(long long, v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__host__ __device__ inline double sg_unord(unsigned long long m) {
    unsigned long long b = (m >> 63) ? (m & 0x7fffffffffffffffull) : ~m;
    return __builtin_bit_cast(double, (long long)b);
}

// ---- launchers (each defined in the translation unit of its kernels) ----
// Scans: exclusive prefix sums of int32 counts into int64 offsets, with
// out[n] = total.  n is read from *n_dev when n_dev != nullptr (device-side
// sizes), else n_host; cap bounds the launch.
size_t sg_scan_tmp_bytes(int64_t cap);
void sg_launch_scan(const int32_t* in, int64_t* out, int64_t n_host, const int64_t* n_dev,
                    int64_t cap, void* tmp, hipStream_t st);

// Gas sort chain.
void sg_launch_grid_reset(sg_grid_dev* g, hipStream_t st);   // keeps the error word
void sg_launch_status_clear(sg_grid_dev* g, hipStream_t st);
void sg_launch_grid_reduce(const double* x, const double* y, const double* z, const double* h,
                           int64_t ng, sg_grid_dev* g, hipStream_t st);
void sg_launch_grid_finish(sg_grid_dev* g, int64_t cell_cap, int cell_scale_log2, hipStream_t st);
void sg_launch_cells_clear(sg_grid_dev* g, int32_t* count, unsigned long long* hmax,
                           int64_t cell_cap, hipStream_t st);
// Cell keys, per-cell counts and max h; also each particle's record
// (x, y, z, h, m) in particle order into pin [ng] (scratch the gather reads).
struct sg_prec;
void sg_launch_keys_count(const double* x, const double* y, const double* z, const double* h,
                          const double* m, int64_t ng, sg_grid_dev* g, int32_t* key,
                          int32_t* count, unsigned long long* hmax, sg_prec* pin,
                          hipStream_t st);
// Stable order of the gas by cell key (ascending id inside a cell): LSD
// radix sort of the keys with 10-bit digits, enough passes for keys below
// cell_cap; tmp: sg_morton_tmp_bytes(ng) bytes.
int sg_gas_radix_passes(int64_t cell_cap);
void sg_launch_gas_order(const int32_t* key, int64_t ng, int64_t cell_cap, void* tmp,
                         int32_t* perm, hipStream_t st);
void sg_launch_gather_gas(const int32_t* perm, int64_t ng, const sg_grid_dev* g,
                          const sg_prec* pin, double* xs, double* ys, double* zs, double* hs,
                          double* ms, sg_prec* prec, hipStream_t st);

// Neighbour lists.
// Neighbour search: per-target slots of fixed length (sg_nbr_slot_bytes),
// counts, then (after the scan and the capacity check) the copy into CSR.
size_t sg_nbr_slot_bytes(int64_t ng);
void sg_launch_nbr_search(const sg_grid_dev* g, int64_t ng, const double* xs, const double* ys,
                          const double* zs, const double* hs, const int64_t* off,
                          const int32_t* perm, const int32_t* key, int32_t* cnt, int32_t* slots,
                          hipStream_t st);
void sg_launch_nbr_check(sg_grid_dev* g, const int64_t* nbr_off, int64_t ng, int64_t nnz_cap,
                         hipStream_t st);
void sg_launch_nbr_compact(const sg_grid_dev* g, int64_t ng, const double* xs, const double* ys,
                           const double* zs, const double* hs, const int64_t* off,
                           const int32_t* cnt, const int32_t* slots, const int64_t* nbr_off,
                           int32_t* nbr_idx, hipStream_t st);

// SPH.  Per-particle data in sorted-slot order is packed into one record
// per particle, so a neighbour gather touches one or two cache lines.
struct alignas(64) sg_prec {          // positions for the density pass
    double x, y, z, h, m, pad[3];
};
struct alignas(32) sg_frec64 {        // FP64 force pass
    double x, y, z, h, m, vx, vy, vz, rho, P, c, pad;   // P = p / rho^2
};
struct alignas(64) sg_frec32 {        // FP32C force pass (FP64 positions)
    double x, y, z;
    float h, m, vx, vy, vz, rho, P, c, pad[2];
};
struct sg_sph_bufs {
    double *xs, *ys, *zs, *hs, *ms;     // sorted SoA (neighbour search, h update)
    double* rho_s;                      // density by slot
    sg_prec* prec;
    sg_frec64* f64;
    sg_frec32* f32;
    const int32_t* perm;
    const int64_t* nbr_off;
    const int32_t* nbr_idx;
    // (vx, vy, vz, e) of each gas particle in particle order, 32 bytes each,
    // packed for the record build's random reads; it borrows the
    // neighbour-search slots, which are free once the lists are copied
    double* ve;
};
void sg_launch_density(const sg_sph_bufs& b, const sg_grid_dev* g, int64_t ng, int precision,
                       double* rho_out, hipStream_t st);
void sg_launch_sph_prep(const sg_sph_bufs& b, const sg_grid_dev* g, int64_t ng, int precision,
                        double gamma, const double* vx, const double* vy, const double* vz,
                        const double* e, hipStream_t st);
// SPH acceleration (asx/asy/asz) and de/dt, both in particle order.
void sg_launch_sph_force(const sg_sph_bufs& b, const sg_grid_dev* g, int64_t ng, int precision,
                         double alpha, double beta, double eta, double* asx, double* asy,
                         double* asz, double* dedt, hipStream_t st);

// Step control: CFL time step into *out (device double) and h update.
void sg_launch_cfl(const sg_sph_bufs& b, const sg_grid_dev* g, int64_t ng, double alpha,
                   double beta, double eta, double C, const double* qx, const double* qy,
                   const double* qz, const double* dedt, double* out, hipStream_t st);
void sg_launch_update_h(const sg_sph_bufs& b, const sg_grid_dev* g, int64_t ng, double sigma,
                        double* h, hipStream_t st);

// Gravity.
struct sg_grav_args {
    const double *x, *y, *z, *m;
    int64_t n;
    double G, eps;
    int precision, ipl, split, with_pot;
    int tile;                           // sources per LDS tile: 128, 256 or 512
    int variant;                        // resolved: FP64 1/2 = difference form with FP32-/FP64-
                                        // seeded rsqrt, 3/4 = expanded far field (Morton order,
                                        // same seeds); FP32C 1 (the only one)
    const int32_t* order;               // FP32C, FP64 3/4: Morton order of the particles
    void* sorted;                       // FP32C, FP64 3/4: scratch of sg_grav_sorted_bytes(n)
    const double *xs, *ys, *zs, *ms;    // (set by the launcher) sorted copies
    const void* sbox;                   // (set by the launcher) sub-tile boxes
    double *gx, *gy, *gz, *gpot;        // outputs [n], particle order
    double* part;                       // split partials [4][split][n] when split > 1
    uint32_t* err;                      // device error word (non-finite positions)
};
size_t sg_grav_sorted_bytes(int64_t n);
// FP32C: Morton-ordered copies of x, y, z, m and the boxes of their
// 64-particle runs (needs a.order and a.sorted); a non-finite position
// sets SGE_GNONFINITE in *a.err.
// Both return -1 (and launch nothing) when a required pointer is missing.
int sg_launch_grav_sorted(const sg_grav_args& a, hipStream_t st);
int sg_launch_gravity(const sg_grav_args& a, hipStream_t st);

// Ensembles: one persistent launch over (system, block of 256*ipl targets)
// tasks of several systems in the FP32C form.
struct sg_ens_sys {
    const double *xs, *ys, *zs, *ms;    // Morton-sorted copies
    const void* sbox;                   // 64-particle boxes
    const int32_t* order;
    int64_t n;
    double *gx, *gy, *gz, *gp;          // outputs, particle order
};
struct sg_ens_task {
    int32_t sys, blk;
};
void sg_grav_sorted_ptrs(void* sorted, int64_t n, const double** xs, const double** ys,
                         const double** zs, const double** ms, const void** sbox);
void sg_launch_grav_ensemble(const sg_ens_sys* d_sys, const sg_ens_task* d_tasks, int32_t ntasks,
                             int32_t* d_counter, int with_pot, double eps, double G, int ipl,
                             int tile, int nblocks, hipStream_t st);
// Workgroups of the ensemble kernel that fit on one CU at once (>= 1).
int sg_grav_ensemble_blocks_per_cu(int ipl, int tile, int with_pot);

// Spatial (Morton) order of all N particles for the FP32C gravity targets.
size_t sg_morton_tmp_bytes(int64_t n);
void sg_launch_morton_order(const double* x, const double* y, const double* z, int64_t n,
                            sg_grid_dev* g, int32_t* order, void* tmp, hipStream_t st);

// Segmented launches: one launch covers a stage for every system of an
// ensemble.  Each system's pointers sit in a device table; a launch's
// blocks are dealt to systems by a prefix of per-system block counts (the
// block of a system is found by a search over that prefix, uniform per
// workgroup).  Each kernel body is the one of the per-system kernel, so
// results are the same bit for bit.
struct sg_seg_sys {
    // caller's state
    double *x, *y, *z, *vx, *vy, *vz, *m, *e, *ax, *ay, *az, *dedt, *rho;
    // workspace: predictor values, SPH and gravity parts
    double *vtx, *vty, *vtz, *et;
    double *asx, *asy, *asz;
    double *gx, *gy, *gz;
    sg_sph_bufs sph;
    sg_grid_dev* g;
    // Morton order: key/value ping-pong buffers, digit histograms and
    // their offsets, the order, sorted copies and 64-particle boxes
    uint32_t *mk0, *mk1;
    int32_t *mv0, *mv1;
    int32_t* mhist;
    int64_t* moffs;
    int32_t* order;
    double *xs, *ys, *zs, *ms;
    void* sbox;
    // gas sort and neighbour lists
    double* h;                       // caller's smoothing lengths
    int32_t *key, *count, *ncnt, *slots;
    // radix sort of the cell keys (as the Morton buffers, for N_g)
    uint32_t *gk0, *gk1;
    int32_t *gv0, *gv1;
    int32_t* ghist;
    int64_t* goffs;
    int64_t gntiles;
    unsigned long long* hmax;
    int64_t* off;
    void* scan;                      // scan scratch (block sums)
    int64_t n, ng, ntiles, cell_cap, nnz_cap;
    double cell_scale;
    double gamma, alpha, beta, eta;
};
// Block prefixes of a segmented launch, per system: blocks of 256
// particles, of 256 gas particles, radix tiles, cell-clearing blocks
// (grid-stride, at most 256 per system), scan tiles of the cell counts and
// of the neighbour counts, blocks of the list copy (sg_compact_blocks),
// radix tiles of the gas, blocks of the SPH density and force passes
// (sg_sph_blocks) and of the neighbour search (sg_nbr_blocks).
enum {
    SG_SEG_N = 0, SG_SEG_NG = 1, SG_SEG_TILES = 2, SG_SEG_CELLS = 3, SG_SEG_SCAN_C = 4,
    SG_SEG_SCAN_G = 5, SG_SEG_CPT = 6, SG_SEG_GTILES = 7, SG_SEG_SPH = 8, SG_SEG_NBR = 9,
    SG_SEG_NPFX = 10
};
struct sg_seg {
    const sg_seg_sys* sys;           // [nsys], device
    const int64_t* pfx;              // [SG_SEG_NPFX][nsys + 1] block prefixes, device
    int32_t nsys;
    int32_t gas_passes;              // radix passes of the cell keys (largest over systems)
    int64_t nblk[SG_SEG_NPFX];       // totals of the prefixes (host)
};
// Host helpers for building the table.
void sg_morton_ptrs(void* tmp, int64_t n, uint32_t** k0, uint32_t** k1, int32_t** v0,
                    int32_t** v1, int32_t** hist, int64_t** offs, int64_t* ntiles);
int64_t sg_radix_tiles(int64_t n);
int64_t sg_scan_tiles(int64_t cap);          // blocks of one sg_launch_scan pass
int64_t sg_cells_clear_blocks(int64_t cell_cap);
// Stages (each one launch, or a few, for all systems).

void sg_seg_launch_combine(const sg_seg& s, hipStream_t st);
void sg_seg_launch_predict(const sg_seg& s, double dt, hipStream_t st);
void sg_seg_launch_correct(const sg_seg& s, double dt, hipStream_t st);
void sg_seg_launch_morton_order(const sg_seg& s, hipStream_t st);
void sg_seg_launch_grav_sorted(const sg_seg& s, hipStream_t st);
// The neighbour build of every system, in the order of the per-system
// launches: the gas sort (grid rule, keys and counts, cell offsets, stable
// reorder and gather), the search, the scan of the neighbour counts into
// CSR offsets, the capacity check and the copy into the CSR rows.
void sg_seg_launch_sort(const sg_seg& s, hipStream_t st);
void sg_seg_launch_nbr_search(const sg_seg& s, hipStream_t st);
void sg_seg_launch_scan_nbr(const sg_seg& s, hipStream_t st);
void sg_seg_launch_nbr_finish(const sg_seg& s, hipStream_t st);
// Density, and the EOS records + FP32C forces on the predicted state
// (predicted != 0: vt, et) or the current one.
int64_t sg_sph_blocks(int64_t ng);
int64_t sg_nbr_blocks(int64_t ng);
int64_t sg_compact_blocks(int64_t ng);
void sg_seg_launch_density(const sg_seg& s, hipStream_t st);
void sg_seg_launch_sph_state(const sg_seg& s, int predicted, hipStream_t st);

// Update and diagnostics.
void sg_launch_predict(int64_t n, int64_t ng, double dt, double* x, double* y, double* z,
                       const double* vx, const double* vy, const double* vz, const double* e,
                       const double* ax, const double* ay, const double* az, const double* dedt,
                       double* vtx, double* vty, double* vtz, double* et, hipStream_t st);
void sg_launch_correct(int64_t n, int64_t ng, double dt, double* vx, double* vy, double* vz,
                       double* e, const double* vtx, const double* vty, const double* vtz,
                       const double* et, const double* ax, const double* ay, const double* az,
                       const double* dedt, hipStream_t st);
void sg_launch_combine(int64_t n, int64_t ng, const double* asx, const double* asy,
                       const double* asz, const double* gx, const double* gy, const double* gz,
                       double* ax, double* ay, double* az, hipStream_t st);
size_t sg_diag_tmp_bytes();
void sg_launch_diagnostics(int64_t n, int64_t ng, const double* x, const double* y,
                           const double* z, const double* vx, const double* vy,
                           const double* vz, const double* m, const double* e,
                           const double* pot, double* tmp, double* out10, hipStream_t st);

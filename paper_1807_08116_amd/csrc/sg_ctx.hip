// sg_ctx.hip -- host side of the C ABI: argument checks, the workspace
// layout, and the order in which the force-evaluation kernels are enqueued
// (the kernel sequence of the paper's predictor-corrector step, Sec. 3).
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "sg_internal.h"

namespace {

thread_local char g_create_msg[256] = "null context";

// grav_variant 0 (automatic) resolved per precision form: FP64 -> 4
// (expanded far field, FP64-seeded rsqrt: 8 % faster than the difference
// form at 2M particles); FP32C has one kernel (1).
constexpr int kAutoVariantFP64 = 4;
inline int resolved_variant(const sg_params& p) {
    if (p.precision == SG_FP32C) return 1;
    return p.grav_variant != 0 ? p.grav_variant : kAutoVariantFP64;
}
// Gravity kernels that work on Morton-ordered copies with per-run boxes.
inline bool uses_morton(const sg_params& p) {
    return p.precision == SG_FP32C || resolved_variant(p) >= 3;
}
// grav_tile 0 (automatic): 256 sources per LDS tile for FP32C, 512 for FP64
// (measured at 2M particles: FP64 2569 ms with 512 against 2640 with 256;
// FP32C best at 256).
inline int resolved_tile(const sg_params& p) {
    if (p.grav_tile != 0) return p.grav_tile;
    return p.precision == SG_FP64 ? 512 : 256;
}

constexpr size_t kAlign = 256;
inline size_t al(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// Largest (split x N) product the automatic gravity launch can ask for.
int64_t part_cap_elems(int64_t n) {
    int64_t a = 64 * n, b = (int64_t(1) << 21) + n;
    return a < b ? a : b;
}

struct layout {
    size_t grid;
    size_t key, perm, gsort;
    size_t count, hmax, off;
    size_t scan;
    size_t xs, ys, zs, hs, ms, rho_s, prec, f64, f32;
    size_t ncnt, nbr_off, nbr_idx, nbr_slots;
    size_t asx, asy, asz;
    size_t gx, gy, gz, gpot;
    size_t gorder, morton, gsorted;
    size_t part;
    size_t vtx, vty, vtz, et;
    size_t diag, diag_out;
    size_t total;
};

layout make_layout(const sg_params* p, const sg_caps* c) {
    layout L;
    const int64_t ng = c->n_gas_cap, n = c->n_gas_cap + c->n_halo_cap;
    const int64_t C = c->cell_cap, Z = c->nnz_cap;
    const bool f32 = p->precision == SG_FP32C;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += al(bytes ? bytes : 1);
        return at;
    };
    L.grid = take(sizeof(sg_grid_dev));
    L.key = take(4 * ng);
    L.perm = take(4 * ng);
    L.gsort = take(sg_morton_tmp_bytes(ng));   // radix sort of the cell keys
    L.count = take(4 * C);
    L.hmax = take(8 * C);
    L.off = take(8 * (C + 1));
    L.scan = take(sg_scan_tmp_bytes(C > ng + 1 ? C : ng + 1));
    size_t* f64s[] = {&L.xs, &L.ys, &L.zs, &L.hs, &L.ms, &L.rho_s};
    for (size_t* q : f64s) *q = take(8 * ng);
    L.prec = take(sizeof(sg_prec) * ng);
    // FP64 force records, also the time-step rule's; between uses the sort
    // borrows the buffer for its particle-order records (64 of 96 bytes)
    L.f64 = take(sizeof(sg_frec64) * ng);
    L.f32 = take(f32 ? sizeof(sg_frec32) * ng : 0);
    L.ncnt = take(4 * ng);
    L.nbr_off = take(8 * (ng + 1));
    L.nbr_idx = take(4 * Z);
    L.nbr_slots = take(sg_nbr_slot_bytes(ng));
    L.asx = take(8 * ng);
    L.asy = take(8 * ng);
    L.asz = take(8 * ng);
    L.gx = take(8 * n);
    L.gy = take(8 * n);
    L.gz = take(8 * n);
    L.gpot = take(8 * n);
    const bool mort = uses_morton(*p);
    L.gorder = take(mort ? 4 * n : 0);
    L.morton = take(mort ? sg_morton_tmp_bytes(n) : 0);
    L.gsorted = take(mort ? sg_grav_sorted_bytes(n) : 0);
    L.part = take(8 * 4 * (size_t)part_cap_elems(n));
    L.vtx = take(8 * n);
    L.vty = take(8 * n);
    L.vtz = take(8 * n);
    L.et = take(8 * ng);
    L.diag = take(sg_diag_tmp_bytes());
    // per-step diagnostics of one captured chunk of steps (sg_run)
    L.diag_out = take(10 * sizeof(double) * (size_t)(p->grav_reorder > 1 ? p->grav_reorder : 1));
    L.total = o;
    return L;
}

bool params_ok(const sg_params* p, const char** why) {
    if (!p) return *why = "params is NULL", false;
    if (!(p->eps > 0.0) || !__builtin_isfinite(p->eps)) return *why = "eps must be > 0", false;
    if (!__builtin_isfinite(p->G)) return *why = "G must be finite", false;
    if (!(p->gamma > 1.0) || !__builtin_isfinite(p->gamma)) return *why = "gamma must be > 1", false;
    if (!(p->alpha >= 0.0) || !(p->beta >= 0.0) || !__builtin_isfinite(p->alpha) ||
        !__builtin_isfinite(p->beta))
        return *why = "alpha, beta must be >= 0", false;
    if (!(p->eta > 0.0) || !__builtin_isfinite(p->eta)) return *why = "eta must be > 0", false;
    if (p->precision != SG_FP64 && p->precision != SG_FP32C)
        return *why = "precision must be SG_FP64 or SG_FP32C", false;
    if (p->grav_ipl != 0 && p->grav_ipl != 1 && p->grav_ipl != 2 && p->grav_ipl != 4)
        return *why = "grav_ipl must be 0, 1, 2 or 4", false;
    if (p->grav_split < 0 || p->grav_split > 64) return *why = "grav_split must be in [0, 64]", false;
    if (p->precision == SG_FP64 && (p->grav_variant < 0 || p->grav_variant > 4))
        return *why = "grav_variant must be 0..4 in the FP64 form", false;
    if (p->precision == SG_FP32C && p->grav_variant != 0 && p->grav_variant != 1)
        return *why = "grav_variant must be 0 or 1 in the FP32C form", false;
    if (p->grav_tile != 0 && p->grav_tile != 128 && p->grav_tile != 256 && p->grav_tile != 512)
        return *why = "grav_tile must be 0, 128, 256 or 512", false;
    if (p->cell_scale_log2 < -1 || p->cell_scale_log2 > 1)
        return *why = "cell_scale_log2 must be -1, 0 or 1", false;
    const int v = resolved_variant(*p);
    if ((v == 1 || v == 3) && !(p->eps * p->eps >= 1.2e-38))
        return *why = "an FP32-seeded reciprocal square root needs eps^2 in the FP32 normal range", false;
    // FP32C forms s = (r^2 + eps^2)^(-3/2) in FP32 before the mass multiplies
    // it (far field); with eps >= 1e-12, s <= 1e36 stays finite, so a
    // massless padding source adds exactly 0
    if (p->precision == SG_FP32C && !(p->eps >= 1e-12))
        return *why = "the FP32C form needs eps >= 1e-12 (finite FP32 (r^2+eps^2)^-1.5)", false;
    if (p->step_serial != 0 && p->step_serial != 1)
        return *why = "step_serial must be 0 or 1", false;
    if (p->grav_reorder < 0 || p->grav_reorder > 1024)
        return *why = "grav_reorder must be in [0, 1024]", false;
    return true;
}

bool caps_ok(const sg_caps* c, const char** why) {
    if (!c) return *why = "caps is NULL", false;
    if (c->n_gas_cap < 0 || c->n_halo_cap < 0 || c->cell_cap < 0 || c->nnz_cap < 0)
        return *why = "capacities must be >= 0", false;
    if (c->n_gas_cap + c->n_halo_cap < 1) return *why = "need room for at least one particle", false;
    if (c->n_gas_cap + c->n_halo_cap > 2147483647ll || c->cell_cap > 2147483646ll)
        return *why = "particle and cell capacities must fit in int32", false;
    if (c->n_gas_cap > 0 && (c->cell_cap < 1 || c->nnz_cap < 1))
        return *why = "gas needs cell_cap >= 1 and nnz_cap >= 1", false;
    return true;
}

}  // namespace

struct sg_ctx {
    sg_params prm;
    sg_caps caps;
    layout L;
    char* ws;
    hipStream_t st;
    // the caller's second stream of a step (gravity beside the
    // neighbour/SPH chain) and the fork / join events between the two;
    // null when no second stream was given or the events could not be
    // created (steps then run their two chains one after the other)
    hipStream_t st2;
    hipEvent_t ev_fork, ev_join;
    // bound state
    bool bound;
    int64_t ng, nh, n;
    sg_state s;
    // validity of cached results for the current positions / velocities
    bool have_nbr, have_rho, have_grav, have_pot, have_sph;
    bool predicted;        // between SG_PREDICT and SG_CORRECT
    bool accel_after_predict;
    // Morton order of the gravity kernels: valid for the bound particles,
    // and gravity preparations since it was computed
    bool have_order;
    int32_t order_age;
    char msg[256];
    // made by sg_create_static: lives in the per-device slot below, over the
    // library's own device array (device index `dev`)
    bool is_static;
    int dev;
    // stage timing
    bool prof;
    struct mark {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<mark> marks;
    std::vector<hipEvent_t> pool;
    double prof_ms[SG_NSTAGE];
    int64_t prof_n[SG_NSTAGE];
    int open_stage;
    hipEvent_t open_ev;

    hipEvent_t take_event() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void begin(int stage) {
        if (!prof) return;
        open_stage = stage;
        open_ev = take_event();
        if (open_ev) (void)hipEventRecord(open_ev, st);
    }
    void end() {
        if (!prof || !open_ev) return;
        hipEvent_t e = take_event();
        if (e) {
            (void)hipEventRecord(e, st);
            marks.push_back(mark{open_stage, open_ev, e});
        }
        open_ev = nullptr;
    }

    template <typename T>
    T* at(size_t off) const {
        return (T*)(ws + off);
    }
    sg_grid_dev* grid() const { return at<sg_grid_dev>(L.grid); }
    sg_status fail(sg_status code, const char* m) {
        snprintf(msg, sizeof(msg), "%s", m);
        return code;
    }
    sg_status check_launch(const char* what) {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            snprintf(msg, sizeof(msg), "%s: %s", what, hipGetErrorString(e));
            return SG_EDEVICE;
        }
        return SG_OK;
    }
    sg_sph_bufs sph() const {
        sg_sph_bufs b;
        b.xs = at<double>(L.xs);
        b.ys = at<double>(L.ys);
        b.zs = at<double>(L.zs);
        b.hs = at<double>(L.hs);
        b.ms = at<double>(L.ms);
        b.rho_s = at<double>(L.rho_s);
        b.prec = at<sg_prec>(L.prec);
        b.f64 = at<sg_frec64>(L.f64);
        b.f32 = at<sg_frec32>(L.f32);
        b.perm = at<int32_t>(L.perm);
        b.nbr_off = at<int64_t>(L.nbr_off);
        b.nbr_idx = at<int32_t>(L.nbr_idx);
        b.ve = at<double>(L.nbr_slots);
        return b;
    }
    void invalidate_positions() {
        have_nbr = have_rho = have_grav = have_pot = have_sph = false;
    }
};

namespace {

sg_status need_bound(sg_ctx* c) {
    if (!c) return SG_EINVAL;
    if (!c->bound) return c->fail(SG_ESTATE, "no state bound (call sg_bind_state)");
    // The runtime's last-error slot is per thread and may hold an error left
    // by another library's earlier call; clear it so that the checks after
    // this entry point's launches see only their own errors.
    (void)hipGetLastError();
    return SG_OK;
}

// Automatic targets per lane: as many as keep enough workgroups to cover
// the 256 CUs several times over.  The FP32C kernel stops at 2: at 4 its
// register footprint (about 200 VGPRs) leaves 2 wavefronts per SIMD, and it
// measured slower than with 2 targets (4 wavefronts per SIMD).
int auto_ipl(int precision, int64_t n) {
    int p = n >= 4 * 256 * 2048 ? 4 : (n >= 2 * 256 * 1024 ? 2 : 1);
    if (precision == SG_FP32C && p > 2) p = 2;
    return p;
}

// Automatic gravity launch shape (targets per lane, source splits).
void grav_shape(const sg_ctx* c, int* ipl, int* split) {
    const int64_t n = c->n;
    int p = c->prm.grav_ipl;
    if (p == 0) p = auto_ipl(c->prm.precision, n);
    int s = c->prm.grav_split;
    const int64_t per = 256 * p;                 // targets per workgroup
    const int64_t iblocks = (n + per - 1) / per;
    if (s == 0) {
        // about 8192 workgroups (32 per CU): measured 4 % faster than 4096
        // for the FP32C kernel at 2M particles, no slower anywhere else
        int64_t want = (8192 + iblocks - 1) / iblocks;
        s = (int)(want < 1 ? 1 : (want > 64 ? 64 : want));
    }
    // the partial buffer bounds split x n
    while (s > 1 && (int64_t)s * n > part_cap_elems(c->caps.n_gas_cap + c->caps.n_halo_cap)) --s;
    *ipl = p;
    *split = s;
}

sg_status do_build(sg_ctx* c) {
    const int64_t ng = c->ng;
    if (ng == 0) {
        c->have_nbr = true;
        return SG_OK;
    }
    hipStream_t st = c->st;
    sg_grid_dev* g = c->grid();
    const sg_state& s = c->s;
    const int64_t C = c->caps.cell_cap;
    int32_t* key = c->at<int32_t>(c->L.key);
    int32_t* count = c->at<int32_t>(c->L.count);
    unsigned long long* hmax = c->at<unsigned long long>(c->L.hmax);
    int64_t* off = c->at<int64_t>(c->L.off);
    void* scan = c->at<void>(c->L.scan);
    sg_sph_bufs b = c->sph();
    c->begin(SG_ST_SORT);
    sg_launch_grid_reset(g, st);
    sg_launch_grid_reduce(s.x, s.y, s.z, s.h, ng, g, st);
    sg_launch_grid_finish(g, C, c->prm.cell_scale_log2, st);
    sg_launch_cells_clear(g, count, hmax, C, st);
    // the FP64 force records are rebuilt before every use (record builds
    // precede each force and time-step pass), so the sort borrows their
    // buffer for the particle-order records the gather reads
    sg_prec* pin = reinterpret_cast<sg_prec*>(b.f64);
    sg_launch_keys_count(s.x, s.y, s.z, s.h, s.m, ng, g, key, count, hmax, pin, st);
    sg_launch_scan(count, off, 0, &g->M, C, scan, st);
    sg_launch_gas_order(key, ng, C, c->at<void>(c->L.gsort), c->at<int32_t>(c->L.perm), st);
    sg_launch_gather_gas(b.perm, ng, g, pin, b.xs, b.ys, b.zs, b.hs, b.ms, b.prec, st);
    c->end();
    c->begin(SG_ST_NBR);
    int32_t* ncnt = c->at<int32_t>(c->L.ncnt);
    int64_t* nbr_off = c->at<int64_t>(c->L.nbr_off);
    int32_t* slots = c->at<int32_t>(c->L.nbr_slots);
    sg_launch_nbr_search(g, ng, b.xs, b.ys, b.zs, b.hs, off, b.perm, key, ncnt, slots, st);
    sg_launch_scan(ncnt, nbr_off, ng, nullptr, ng, scan, st);
    sg_launch_nbr_check(g, nbr_off, ng, c->caps.nnz_cap, st);
    sg_launch_nbr_compact(g, ng, b.xs, b.ys, b.zs, b.hs, off, ncnt, slots, nbr_off,
                          c->at<int32_t>(c->L.nbr_idx), st);
    c->end();
    sg_status r = c->check_launch("neighbour build");
    if (r != SG_OK) return r;
    c->have_nbr = true;
    c->have_rho = false;
    return SG_OK;
}

sg_status do_density(sg_ctx* c) {
    if (c->ng > 0) {
        if (!c->have_nbr) return c->fail(SG_ESTATE, "density needs neighbour lists");
        c->begin(SG_ST_DENSITY);
        sg_launch_density(c->sph(), c->grid(), c->ng, c->prm.precision, c->s.rho, c->st);
        c->end();
        sg_status r = c->check_launch("density");
        if (r != SG_OK) return r;
    }
    c->have_rho = true;
    return SG_OK;
}

void grav_args(sg_ctx* c, bool pot, sg_grav_args& a) {
    a.x = c->s.x;
    a.y = c->s.y;
    a.z = c->s.z;
    a.m = c->s.m;
    a.n = c->n;
    a.G = c->prm.G;
    a.eps = c->prm.eps;
    a.precision = c->prm.precision;
    grav_shape(c, &a.ipl, &a.split);
    a.tile = resolved_tile(c->prm);
    a.with_pot = pot ? 1 : 0;
    a.variant = resolved_variant(c->prm);
    a.order = uses_morton(c->prm) ? c->at<int32_t>(c->L.gorder) : nullptr;
    a.sorted = c->at<void>(c->L.gsorted);
    a.gx = c->at<double>(c->L.gx);
    a.gy = c->at<double>(c->L.gy);
    a.gz = c->at<double>(c->L.gz);
    a.gpot = c->s.pot ? c->s.pot : c->at<double>(c->L.gpot);
    a.part = c->at<double>(c->L.part);
    a.err = &c->grid()->err;
}

// Gravity preparations per Morton sort (1 when the kernel uses no order).
int reorder_period(const sg_ctx* c) {
    return uses_morton(c->prm) && c->prm.grav_reorder > 1 ? c->prm.grav_reorder : 1;
}

// The next gravity preparation recomputes the Morton order.
bool sorts_next(const sg_ctx* c) {
    return !c->have_order || c->order_age >= reorder_period(c);
}

// Morton order, sorted copies and 64-particle boxes at the current
// positions (FP32C and the FP64 expanded-far-field kernels only).
sg_status grav_prep(sg_ctx* c, const sg_grav_args& a) {
    if (!uses_morton(c->prm)) return SG_OK;
    c->begin(SG_ST_GRAV_PREP);
    if (sorts_next(c)) {
        sg_launch_morton_order(c->s.x, c->s.y, c->s.z, c->n, c->grid(),
                               const_cast<int32_t*>(a.order), c->at<void>(c->L.morton), c->st);
        c->have_order = true;
        c->order_age = 0;
    }
    ++c->order_age;
    const int rc = sg_launch_grav_sorted(a, c->st);
    c->end();
    if (rc != 0) return c->fail(SG_EINVAL, "gravity preparation: missing buffer");
    return SG_OK;
}

sg_status do_gravity(sg_ctx* c, bool pot) {
    sg_grav_args a;
    grav_args(c, pot, a);
    sg_status r = grav_prep(c, a);
    if (r != SG_OK) return r;
    c->begin(SG_ST_GRAV);
    const int rc = sg_launch_gravity(a, c->st);
    c->end();
    if (rc != 0) return c->fail(SG_EINVAL, "gravity: missing buffer");
    if ((r = c->check_launch("gravity")) != SG_OK) return r;
    c->have_grav = true;
    c->have_pot = pot;
    return SG_OK;
}

sg_status do_sph(sg_ctx* c) {
    if (c->ng == 0) {
        c->have_sph = true;
        return SG_OK;
    }
    if (!c->have_rho) return c->fail(SG_ESTATE, "SPH forces need the density");
    const double* vx = c->predicted ? c->at<double>(c->L.vtx) : c->s.vx;
    const double* vy = c->predicted ? c->at<double>(c->L.vty) : c->s.vy;
    const double* vz = c->predicted ? c->at<double>(c->L.vtz) : c->s.vz;
    const double* e = c->predicted ? c->at<double>(c->L.et) : c->s.e;
    sg_sph_bufs b = c->sph();
    c->begin(SG_ST_SPH);
    sg_launch_sph_prep(b, c->grid(), c->ng, c->prm.precision, c->prm.gamma, vx, vy, vz, e, c->st);
    sg_launch_sph_force(b, c->grid(), c->ng, c->prm.precision, c->prm.alpha, c->prm.beta,
                        c->prm.eta, c->at<double>(c->L.asx), c->at<double>(c->L.asy),
                        c->at<double>(c->L.asz), c->s.dedt, c->st);
    c->end();
    sg_status r = c->check_launch("SPH forces");
    if (r != SG_OK) return r;
    c->have_sph = true;
    return SG_OK;
}

void do_combine(sg_ctx* c) {
    const bool sph = c->have_sph && c->ng > 0;
    c->begin(SG_ST_UPDATE);
    sg_launch_combine(c->n, c->ng, sph ? c->at<double>(c->L.asx) : nullptr,
                      sph ? c->at<double>(c->L.asy) : nullptr,
                      sph ? c->at<double>(c->L.asz) : nullptr,
                      c->have_grav ? c->at<double>(c->L.gx) : nullptr,
                      c->have_grav ? c->at<double>(c->L.gy) : nullptr,
                      c->have_grav ? c->at<double>(c->L.gz) : nullptr, c->s.ax, c->s.ay, c->s.az,
                      c->st);
    c->end();
}

sg_status do_accel(sg_ctx* c, uint32_t flags) {
    if (flags & ~(SG_SPH | SG_GRAV | SG_POT)) return c->fail(SG_EINVAL, "unknown flags");
    if ((flags & SG_POT) && !(flags & SG_GRAV)) return c->fail(SG_EINVAL, "SG_POT needs SG_GRAV");
    sg_status r;
    if (flags & SG_GRAV) {
        if ((r = do_gravity(c, (flags & SG_POT) != 0)) != SG_OK) return r;
    }
    if (flags & SG_SPH) {
        if ((r = do_sph(c)) != SG_OK) return r;
    }
    do_combine(c);
    if (c->predicted) c->accel_after_predict = true;
    return c->check_launch("combine");
}

sg_status do_kick_drift(sg_ctx* c, double dt, int phase) {
    if (!__builtin_isfinite(dt)) return c->fail(SG_EINVAL, "dt must be finite");
    const sg_state& s = c->s;
    double* vtx = c->at<double>(c->L.vtx);
    double* vty = c->at<double>(c->L.vty);
    double* vtz = c->at<double>(c->L.vtz);
    double* et = c->at<double>(c->L.et);
    if (phase == SG_PREDICT) {
        if (c->predicted) return c->fail(SG_ESTATE, "SG_PREDICT twice without SG_CORRECT");
        if (!c->have_grav || !(c->have_sph || c->ng == 0))
            return c->fail(SG_ESTATE, "SG_PREDICT needs gravity and SPH forces at the current state");
        c->begin(SG_ST_UPDATE);
        sg_launch_predict(c->n, c->ng, dt, s.x, s.y, s.z, s.vx, s.vy, s.vz, s.e, s.ax, s.ay, s.az,
                          s.dedt, vtx, vty, vtz, et, c->st);
        c->end();
        c->invalidate_positions();
        c->predicted = true;
        c->accel_after_predict = false;
    } else if (phase == SG_CORRECT) {
        if (!c->predicted) return c->fail(SG_ESTATE, "SG_CORRECT without SG_PREDICT");
        if (!c->accel_after_predict || !c->have_grav || !(c->have_sph || c->ng == 0))
            return c->fail(SG_ESTATE, "SG_CORRECT needs gravity and SPH forces after SG_PREDICT");
        c->begin(SG_ST_UPDATE);
        sg_launch_correct(c->n, c->ng, dt, s.vx, s.vy, s.vz, s.e, vtx, vty, vtz, et, s.ax, s.ay,
                          s.az, s.dedt, c->st);
        c->end();
        c->predicted = false;
        c->have_sph = false;       // the SPH part was evaluated with the predicted velocities
    } else {
        return c->fail(SG_EINVAL, "phase must be SG_PREDICT or SG_CORRECT");
    }
    return c->check_launch("kick/drift");
}


sg_status do_step(sg_ctx* c, double dt, uint32_t flags) {
    sg_status r;
    if (flags & ~SG_POT) return c->fail(SG_EINVAL, "steps accept only SG_POT");
    if (!__builtin_isfinite(dt)) return c->fail(SG_EINVAL, "dt must be finite");
    if (c->predicted) return c->fail(SG_ESTATE, "step inside a predict/correct pair");
    const uint32_t gflags = SG_GRAV | (flags & SG_POT);
    // forces at r(t): neighbours and density are reused from the previous
    // step's corrector (positions unchanged since), gravity likewise.
    if (!c->have_nbr && (r = do_build(c)) != SG_OK) return r;
    if (!c->have_rho && (r = do_density(c)) != SG_OK) return r;
    if (!c->have_grav || ((flags & SG_POT) && !c->have_pot))
        if ((r = do_gravity(c, (flags & SG_POT) != 0)) != SG_OK) return r;
    if ((r = do_sph(c)) != SG_OK) return r;                 // predictor right-hand side
    do_combine(c);
    if ((r = do_kick_drift(c, dt, SG_PREDICT)) != SG_OK) return r;
    // corrector right-hand side.  Gravity at the predicted positions and the
    // neighbour build -> density -> SPH forces chain are independent: with a
    // second stream, the chain runs there (forked from the context's stream
    // before the gravity is enqueued on it, and joined back, also while the
    // stream is being captured).  They touch disjoint workspace buffers and
    // disjoint fields of the grid record (the status word by atomic OR).
    // Gravity first on the context's stream: measured on ensembles, the
    // persistent gravity kernel keeps its pace when its workgroups are
    // dispatched ahead of the chain's, and loses 14 % when the chain's come
    // first.
    if (!c->st2 || c->prm.step_serial) {
        if ((r = do_build(c)) != SG_OK) return r;
        if ((r = do_density(c)) != SG_OK) return r;
        if ((r = do_accel(c, gflags | SG_SPH)) != SG_OK) return r;
        return do_kick_drift(c, dt, SG_CORRECT);
    }
    if (hipEventRecord(c->ev_fork, c->st) != hipSuccess ||
        hipStreamWaitEvent(c->st2, c->ev_fork, 0) != hipSuccess)
        return c->fail(SG_EDEVICE, "step: fork to the second stream failed");
    sg_status rg = do_gravity(c, (flags & SG_POT) != 0);
    hipStream_t own = c->st;
    c->st = c->st2;
    sg_status rs = rg != SG_OK ? rg : do_build(c);
    if (rs == SG_OK) rs = do_density(c);
    if (rs == SG_OK) rs = do_sph(c);
    c->st = own;
    // join (also after an error, so that a capture stays whole)
    if ((hipEventRecord(c->ev_join, c->st2) != hipSuccess ||
         hipStreamWaitEvent(c->st, c->ev_join, 0) != hipSuccess) && rs == SG_OK)
        rs = c->fail(SG_EDEVICE, "step: join of the second stream failed");
    if (rs != SG_OK) return rs;
    do_combine(c);
    c->accel_after_predict = true;
    if ((r = c->check_launch("combine")) != SG_OK) return r;
    return do_kick_drift(c, dt, SG_CORRECT);
}

sg_status do_diag(sg_ctx* c, double* d_out10) {
    const double* pot = nullptr;
    if (c->have_pot) pot = c->s.pot ? c->s.pot : c->at<double>(c->L.gpot);
    c->begin(SG_ST_DIAG);
    sg_launch_diagnostics(c->n, c->ng, c->s.x, c->s.y, c->s.z, c->s.vx, c->s.vy, c->s.vz, c->s.m,
                          c->s.e, pot, c->at<double>(c->L.diag), d_out10, c->st);
    c->end();
    return c->check_launch("diagnostics");
}

// Everything sg_create and sg_create_static share: fields, the cleared
// status word and grid record (the workspace may hold anything).
sg_status init_ctx(sg_ctx* c, const sg_params* prm, const sg_caps* caps, const layout& L,
                   char* ws, hipStream_t stream) {
    c->prm = *prm;
    c->caps = *caps;
    c->L = L;
    c->ws = ws;
    c->st = stream;
    c->bound = false;
    c->ng = c->nh = c->n = 0;
    memset(&c->s, 0, sizeof(c->s));
    c->invalidate_positions();
    c->have_order = false;
    c->order_age = 0;
    c->predicted = false;
    c->accel_after_predict = false;
    c->msg[0] = 0;
    c->prof = false;
    c->open_ev = nullptr;
    c->open_stage = 0;
    for (int k = 0; k < SG_NSTAGE; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_n[k] = 0;
    }
    (void)hipGetLastError();            // drop a stale error of an earlier call
    sg_launch_status_clear(c->grid(), c->st);
    sg_launch_grid_reset(c->grid(), c->st);
    return c->check_launch("create");
}

}  // namespace

// ------------------------------------------------ allocation-free contexts --
// The workspace of contexts made by sg_create_static: one file-scope device
// array, of which the runtime gives every GPU the library runs on its own
// copy, held until the process ends.  Host code never passes the array's
// name to the GPU (on the host it only stands for the symbol): its device
// address on the current GPU comes from hipGetSymbolAddress, once per
// device, and only that address is used.
static __device__ __attribute__((aligned(256))) char scratch[SG_STATIC_WS_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
char* g_static_ptr[kMaxDevices];      // device address of `scratch`, per device
bool g_static_live[kMaxDevices];      // a static context exists on the device
sg_ctx g_static_ctx[kMaxDevices];     // its host record (no allocation)

// Claim the current device's array (its address resolved on first use).
sg_status static_acquire(int* dev_out, char** ws_out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
        snprintf(g_create_msg, sizeof(g_create_msg), "no current HIP device");
        return SG_EDEVICE;
    }
    if (dev >= kMaxDevices) {
        snprintf(g_create_msg, sizeof(g_create_msg), "device index beyond %d", kMaxDevices - 1);
        return SG_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_live[dev]) {
        snprintf(g_create_msg, sizeof(g_create_msg),
                 "a static context already exists on device %d (destroy it first)", dev);
        return SG_ESTATE;
    }
    if (!g_static_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            snprintf(g_create_msg, sizeof(g_create_msg), "hipGetSymbolAddress: %s",
                     hipGetErrorString(e));
            (void)hipGetLastError();
            return SG_EDEVICE;
        }
        g_static_ptr[dev] = (char*)p;
    }
    g_static_live[dev] = true;
    *dev_out = dev;
    *ws_out = g_static_ptr[dev];
    return SG_OK;
}

void static_release(int dev) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static_live[dev] = false;
}

}  // namespace

extern "C" {

size_t sg_workspace_bytes(const sg_params* prm, const sg_caps* caps) {
    const char* why;
    if (!params_ok(prm, &why) || !caps_ok(caps, &why)) return 0;
    return make_layout(prm, caps).total;
}

sg_status sg_create(const sg_params* prm, const sg_caps* caps, void* d_workspace,
                    size_t ws_bytes, void* stream, void* aux_stream, sg_ctx** out) {
    if (!out) return SG_EINVAL;
    *out = nullptr;
    const char* why = nullptr;
    if (!params_ok(prm, &why) || !caps_ok(caps, &why)) {
        snprintf(g_create_msg, sizeof(g_create_msg), "%s", why ? why : "invalid arguments");
        return SG_EINVAL;
    }
    if (!d_workspace || ((uintptr_t)d_workspace & (kAlign - 1))) {
        snprintf(g_create_msg, sizeof(g_create_msg), "workspace must be 256-byte aligned, non-null");
        return SG_EINVAL;
    }
    layout L = make_layout(prm, caps);
    if (ws_bytes < L.total) {
        snprintf(g_create_msg, sizeof(g_create_msg), "workspace smaller than sg_workspace_bytes()");
        return SG_EINVAL;
    }
    sg_ctx* c = new (std::nothrow) sg_ctx();
    if (!c) return SG_EINVAL;
    c->ev_fork = c->ev_join = nullptr;
    c->st2 = nullptr;
    if (aux_stream && aux_stream != stream) {
        if (hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
            // without them, steps run their two chains one after the other
            if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
            c->ev_fork = c->ev_join = nullptr;
        } else {
            c->st2 = (hipStream_t)aux_stream;
        }
    }
    if (init_ctx(c, prm, caps, L, (char*)d_workspace, (hipStream_t)stream) != SG_OK) {
        snprintf(g_create_msg, sizeof(g_create_msg), "%s", c->msg);
        if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
        if (c->ev_join) (void)hipEventDestroy(c->ev_join);
        delete c;
        return SG_EDEVICE;
    }
    *out = c;
    return SG_OK;
}

sg_status sg_create_static(const sg_params* prm, const sg_caps* caps, void* stream,
                           sg_ctx** out) {
    if (!out) return SG_EINVAL;
    *out = nullptr;
    const char* why = nullptr;
    if (!params_ok(prm, &why) || !caps_ok(caps, &why)) {
        snprintf(g_create_msg, sizeof(g_create_msg), "%s", why ? why : "invalid arguments");
        return SG_EINVAL;
    }
    const layout L = make_layout(prm, caps);
    if (L.total > (size_t)SG_STATIC_WS_BYTES) {
        snprintf(g_create_msg, sizeof(g_create_msg),
                 "workspace of %zu bytes for these capacities exceeds the static array (%llu bytes)",
                 L.total, (unsigned long long)SG_STATIC_WS_BYTES);
        return SG_ECAPACITY;
    }
    char* ws = nullptr;
    int dev = -1;
    sg_status r = static_acquire(&dev, &ws);
    if (r != SG_OK) return r;
    sg_ctx* c = &g_static_ctx[dev];
    c->st2 = nullptr;                 // one stream, no events: steps run in order
    c->ev_fork = c->ev_join = nullptr;
    c->is_static = true;
    c->dev = dev;
    if (init_ctx(c, prm, caps, L, ws, (hipStream_t)stream) != SG_OK) {
        snprintf(g_create_msg, sizeof(g_create_msg), "%s", c->msg);
        static_release(dev);
        return SG_EDEVICE;
    }
    *out = c;
    return SG_OK;
}

sg_status sg_bind_state(sg_ctx* c, int64_t n_gas, int64_t n_halo, const sg_state* st) {
    if (!c) return SG_EINVAL;
    (void)hipGetLastError();
    if (!st) return c->fail(SG_EINVAL, "state is NULL");
    if (n_gas < 0 || n_halo < 0 || n_gas + n_halo < 1)
        return c->fail(SG_EINVAL, "need n_gas, n_halo >= 0 and at least one particle");
    if (n_gas > c->caps.n_gas_cap || n_halo > c->caps.n_halo_cap)
        return c->fail(SG_EINVAL, "particle counts exceed the capacities");
    if (!st->x || !st->y || !st->z || !st->vx || !st->vy || !st->vz || !st->m || !st->ax ||
        !st->ay || !st->az)
        return c->fail(SG_EINVAL, "a required state pointer is NULL");
    if (n_gas > 0 && (!st->h || !st->e || !st->dedt || !st->rho))
        return c->fail(SG_EINVAL, "gas needs h, e, dedt and rho");
    const void* ptrs[] = {st->x, st->y, st->z, st->vx, st->vy, st->vz, st->m, st->ax, st->ay,
                          st->az, st->h, st->e, st->dedt, st->rho, st->pot};
    for (const void* p : ptrs)
        if (p && ((uintptr_t)p & 7)) return c->fail(SG_EINVAL, "state pointers must be 8-byte aligned");
    c->s = *st;
    c->ng = n_gas;
    c->nh = n_halo;
    c->n = n_gas + n_halo;
    c->bound = true;
    c->invalidate_positions();
    c->have_order = false;
    c->predicted = false;
    c->accel_after_predict = false;
    sg_launch_status_clear(c->grid(), c->st);
    return c->check_launch("bind");
}

sg_status sg_build_neighbors(sg_ctx* c) {
    sg_status r = need_bound(c);
    return r != SG_OK ? r : do_build(c);
}

sg_status sg_compute_density(sg_ctx* c) {
    sg_status r = need_bound(c);
    return r != SG_OK ? r : do_density(c);
}

sg_status sg_compute_accel(sg_ctx* c, uint32_t flags) {
    sg_status r = need_bound(c);
    if (r != SG_OK) return r;
    return do_accel(c, flags);
}

sg_status sg_kick_drift(sg_ctx* c, double dt, int32_t phase) {
    sg_status r = need_bound(c);
    return r != SG_OK ? r : do_kick_drift(c, dt, phase);
}

sg_status sg_step(sg_ctx* c, double dt, uint32_t flags) {
    sg_status r = need_bound(c);
    return r != SG_OK ? r : do_step(c, dt, flags);
}

sg_status sg_run(sg_ctx* c, double dt, int64_t nsteps, uint32_t flags, int32_t use_graph,
                 double* d_hist) {
    sg_status r = need_bound(c);
    if (r != SG_OK) return r;
    if (nsteps < 0) return c->fail(SG_EINVAL, "nsteps must be >= 0");
    if (use_graph && c->prof) return c->fail(SG_ESTATE, "stage timing must be off to capture a graph");
    if (use_graph && nsteps >= 2 && c->st == nullptr)
        return c->fail(SG_EINVAL, "graph capture needs a stream other than the null stream");
    double* diag = c->at<double>(c->L.diag_out);
    // A captured chunk holds one period of the Morton-order schedule (P
    // steps, one recomputation each), so that its replays recompute the
    // order exactly where eager steps would.
    const int64_t P = reorder_period(c);
    auto eager = [&](int64_t k) {
        sg_status q = do_step(c, dt, flags);
        if (q == SG_OK && d_hist) q = do_diag(c, d_hist + 10 * k);
        return q;
    };
    int64_t k = 0;
    const int64_t chunks = nsteps >= 1 ? (nsteps - 1) / P : 0;
    if (!use_graph || chunks < 1) {
        for (; k < nsteps; ++k)
            if ((r = eager(k)) != SG_OK) return r;
        return hipStreamSynchronize(c->st) == hipSuccess ? SG_OK
                                                          : c->fail(SG_EDEVICE, "stream sync failed");
    }
    // one eager step reaches the steady state (cached lists and forces)
    if ((r = eager(k++)) != SG_OK) return r;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (hipStreamBeginCapture(c->st, hipStreamCaptureModeRelaxed) != hipSuccess)
        return c->fail(SG_EDEVICE, "hipStreamBeginCapture failed");
    sg_status rc = SG_OK;
    for (int64_t j = 0; j < P && rc == SG_OK; ++j) {
        rc = do_step(c, dt, flags);
        if (rc == SG_OK && d_hist) rc = do_diag(c, diag + 10 * j);
    }
    hipError_t ec = hipStreamEndCapture(c->st, &graph);
    if (rc != SG_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (ec != hipSuccess || !graph) return c->fail(SG_EDEVICE, "hipStreamEndCapture failed");
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return c->fail(SG_EDEVICE, "hipGraphInstantiate failed");
    }
    for (int64_t q = 0; q < chunks && rc == SG_OK; ++q, k += P) {
        if (hipGraphLaunch(exec, c->st) != hipSuccess) rc = c->fail(SG_EDEVICE, "hipGraphLaunch failed");
        else if (d_hist && hipMemcpyAsync(d_hist + 10 * k, diag, 10 * sizeof(double) * (size_t)P,
                                          hipMemcpyDeviceToDevice, c->st) != hipSuccess)
            rc = c->fail(SG_EDEVICE, "history copy failed");
    }
    for (; k < nsteps && rc == SG_OK; ++k) rc = eager(k);
    if (hipStreamSynchronize(c->st) != hipSuccess && rc == SG_OK)
        rc = c->fail(SG_EDEVICE, "stream sync failed");
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return rc;
}

sg_status sg_cfl_dt(sg_ctx* c, double C, double* d_dt) {
    sg_status r = need_bound(c);
    if (r != SG_OK) return r;
    if (!d_dt || ((uintptr_t)d_dt & 7)) return c->fail(SG_EINVAL, "d_dt must be an aligned device pointer");
    if (!(C > 0.0) || !__builtin_isfinite(C)) return c->fail(SG_EINVAL, "C must be > 0");
    if (c->ng == 0) return c->fail(SG_ESTATE, "the time-step rule needs gas particles");
    if (c->predicted) return c->fail(SG_ESTATE, "time step inside a predict/correct pair");
    if (!c->have_rho || !c->have_grav || !c->have_sph)
        return c->fail(SG_ESTATE, "time step needs neighbours, density and accelerations");
    sg_sph_bufs b = c->sph();
    // sound speeds and velocities of the current state, FP64, slot order
    sg_launch_sph_prep(b, c->grid(), c->ng, SG_FP64, c->prm.gamma, c->s.vx, c->s.vy, c->s.vz,
                       c->s.e, c->st);
    sg_launch_cfl(b, c->grid(), c->ng, c->prm.alpha, c->prm.beta, c->prm.eta, C, c->s.ax, c->s.ay,
                  c->s.az, c->s.dedt, d_dt, c->st);
    return c->check_launch("time step");
}

sg_status sg_update_h(sg_ctx* c, double sigma) {
    sg_status r = need_bound(c);
    if (r != SG_OK) return r;
    if (!(sigma > 0.0) || !__builtin_isfinite(sigma)) return c->fail(SG_EINVAL, "sigma must be > 0");
    if (c->predicted) return c->fail(SG_ESTATE, "h update inside a predict/correct pair");
    if (c->ng == 0) return SG_OK;
    if (!c->have_rho) return c->fail(SG_ESTATE, "h update needs the density");
    sg_launch_update_h(c->sph(), c->grid(), c->ng, sigma, c->s.h, c->st);
    c->invalidate_positions();     // lists, density and forces depend on h
    return c->check_launch("h update");
}

sg_status sg_diagnostics(sg_ctx* c, double* d_out10) {
    sg_status r = need_bound(c);
    if (r != SG_OK) return r;
    if (!d_out10) return c->fail(SG_EINVAL, "output is NULL");
    return do_diag(c, d_out10);
}

sg_status sg_export(sg_ctx* c, int32_t what, void* dst, int64_t cap_bytes, int64_t* n_out) {
    sg_status r = need_bound(c);
    if (r != SG_OK) return r;
    if (!dst || !n_out) return c->fail(SG_EINVAL, "destination or n_out is NULL");
    if (hipStreamSynchronize(c->st) != hipSuccess) return c->fail(SG_EDEVICE, "stream sync failed");
    sg_grid_dev g;
    if (hipMemcpy(&g, c->grid(), sizeof(g), hipMemcpyDeviceToHost) != hipSuccess)
        return c->fail(SG_EDEVICE, "reading the grid failed");
    const int64_t ng = c->ng, M = g.M;
    const void* src = nullptr;
    int64_t n = 0, esz = 0;
    switch (what) {
        case SG_X_KEYS: src = c->at<void>(c->L.key); n = ng; esz = 4; break;
        case SG_X_COUNTS: src = c->at<void>(c->L.count); n = M; esz = 4; break;
        case SG_X_OFFSETS: src = c->at<void>(c->L.off); n = M + 1; esz = 8; break;
        case SG_X_HMAX: src = c->at<void>(c->L.hmax); n = M; esz = 8; break;
        case SG_X_PERM: src = c->at<void>(c->L.perm); n = ng; esz = 4; break;
        case SG_X_NBR_OFF: src = c->at<void>(c->L.nbr_off); n = ng + 1; esz = 8; break;
        case SG_X_NBR_IDX: src = c->at<void>(c->L.nbr_idx); n = g.nnz; esz = 4; break;
        case SG_X_GORDER:
            if (!uses_morton(c->prm)) return c->fail(SG_EINVAL, "no gravity order for this kernel");
            src = c->at<void>(c->L.gorder); n = c->n; esz = 4; break;
        case SG_X_ACC_SPH:
        case SG_X_ACC_GRAV: {
            // three component arrays, copied one after the other
            const bool sph = what == SG_X_ACC_SPH;
            if (sph ? !c->have_sph : !c->have_grav)
                return c->fail(SG_ESTATE, sph ? "no SPH acceleration computed yet"
                                              : "no gravity computed yet");
            const int64_t len = sph ? ng : c->n;
            *n_out = 3 * len;
            if (3 * len * 8 > cap_bytes) return c->fail(SG_ECAPACITY, "destination too small");
            const size_t part[3] = {sph ? c->L.asx : c->L.gx, sph ? c->L.asy : c->L.gy,
                                    sph ? c->L.asz : c->L.gz};
            for (int d = 0; d < 3 && len > 0; ++d)
                if (hipMemcpy(static_cast<char*>(dst) + (size_t)d * len * 8, c->at<void>(part[d]),
                              (size_t)len * 8, hipMemcpyDeviceToDevice) != hipSuccess)
                    return c->fail(SG_EDEVICE, "export copy failed");
            return SG_OK;
        }
        case SG_X_GRID: {
            if (cap_bytes < (int64_t)sizeof(sg_grid_info)) return c->fail(SG_ECAPACITY, "buffer too small");
            sg_grid_info info;
            memset(&info, 0, sizeof(info));
            info.L0 = g.L0;
            info.nlev = g.nlev;
            for (int l = 0; l < SG_MAXLEV; ++l) {
                info.L[l] = g.L[l];
                info.base[l] = g.base[l];
                info.ncell[l] = g.ncell[l];
                info.npart[l] = (int64_t)g.npart[l];
                info.hmax[l] = g.hmaxlev[l];
                for (int d = 0; d < 3; ++d) {
                    info.org[l][d] = g.org[l][d];
                    info.dim[l][d] = g.dim[l][d];
                }
            }
            info.M = g.M;
            memcpy(dst, &info, sizeof(info));
            *n_out = 1;
            return SG_OK;
        }
        default: return c->fail(SG_EINVAL, "unknown export");
    }
    *n_out = n;
    if (n * esz > cap_bytes) return c->fail(SG_ECAPACITY, "destination too small");
    if (n > 0 && hipMemcpy(dst, src, (size_t)(n * esz), hipMemcpyDeviceToDevice) != hipSuccess)
        return c->fail(SG_EDEVICE, "export copy failed");
    return SG_OK;
}

sg_status sg_status_sync(sg_ctx* c, int64_t need[2]) {
    if (!c) return SG_EINVAL;
    if (hipStreamSynchronize(c->st) != hipSuccess) return c->fail(SG_EDEVICE, "stream sync failed");
    sg_grid_dev g;
    if (hipMemcpy(&g, c->grid(), sizeof(g), hipMemcpyDeviceToHost) != hipSuccess)
        return c->fail(SG_EDEVICE, "reading the status failed");
    if (need) {
        need[0] = g.need_cells;
        need[1] = g.need_nnz;
    }
    if (g.err == 0) return SG_OK;
    sg_launch_status_clear(c->grid(), c->st);
    (void)hipStreamSynchronize(c->st);
    c->invalidate_positions();
    if (g.err & (SGE_NONFINITE | SGE_GNONFINITE))
        return c->fail(SG_ENONFINITE, "non-finite position or smoothing length <= 0");
    if (g.err & SGE_LEVELS)
        return c->fail(SG_ERANGE, "smoothing lengths span more than SG_MAX_LEVELS levels");
    if (g.err & SGE_GRID) return c->fail(SG_ERANGE, "grid level too large for int32 cell keys");
    snprintf(c->msg, sizeof(c->msg), "capacity exceeded: need %lld cells, %lld neighbour pairs",
             (long long)g.need_cells, (long long)g.need_nnz);
    return SG_ECAPACITY;
}

// ------------------------------------------------------------- ensembles --

struct sg_ens {
    std::vector<sg_ctx*> c;
    hipStream_t st;
    // the stream of the systems' corrector chains beside the batched
    // gravity, with its fork/join events: the caller's, or one the ensemble
    // creates with every CU in its mask (which gives it a hardware queue of
    // its own; own_cst)
    hipStream_t cst;
    bool own_cst;
    hipEvent_t cev[2];
    sg_ens_sys* d_sys;
    sg_ens_task* d_tasks;
    int32_t* d_counter;
    int32_t ntasks;
    int nblocks, ipl, tile;
    double eps, G;
    sg_seg seg;                  // segmented launches over all systems
    char msg[256];
    sg_status fail(sg_status code, const char* m) {
        snprintf(msg, sizeof(msg), "%s", m);
        return code;
    }
    ~sg_ens() {
        if (st) (void)hipStreamSynchronize(st);
        if (cst) (void)hipStreamSynchronize(cst);
        if (cst && own_cst) (void)hipStreamDestroy(cst);
        for (hipEvent_t x : cev)
            if (x) (void)hipEventDestroy(x);
    }
};

extern "C++" {
namespace {

struct ens_offsets {
    size_t tasks, counter, seg, pfx, total;
};

ens_offsets ens_layout(int32_t nsys, int64_t ntasks) {
    ens_offsets o;
    size_t at = al(sizeof(sg_ens_sys) * (size_t)nsys);
    o.tasks = at;
    at += al(sizeof(sg_ens_task) * (size_t)(ntasks > 0 ? ntasks : 1));
    o.counter = at;
    at += al(sizeof(int32_t));
    o.seg = at;
    at += al(sizeof(sg_seg_sys) * (size_t)nsys);
    o.pfx = at;
    at += al(sizeof(int64_t) * SG_SEG_NPFX * (size_t)(nsys + 1));
    o.total = at;
    return o;
}

// Morton order (when due) and sorted copies of every system, in segmented
// launches on the shared stream.  The systems of an ensemble normally share
// the schedule of the order; a system whose schedule differs (it was
// stepped on its own) gets its own sort.
sg_status ens_grav_prep(sg_ens* e) {
    sg_ctx* c0 = e->c[0];
    c0->begin(SG_ST_GRAV_PREP);
    bool all = true;
    for (sg_ctx* c : e->c) all = all && sorts_next(c);
    if (all) sg_seg_launch_morton_order(e->seg, e->st);
    for (sg_ctx* c : e->c) {
        if (sorts_next(c)) {
            if (!all)
                sg_launch_morton_order(c->s.x, c->s.y, c->s.z, c->n, c->grid(),
                                       c->at<int32_t>(c->L.gorder), c->at<void>(c->L.morton), e->st);
            c->have_order = true;
            c->order_age = 0;
        }
        ++c->order_age;
    }
    sg_seg_launch_grav_sorted(e->seg, e->st);
    c0->end();
    hipError_t err = hipGetLastError();
    return err == hipSuccess ? SG_OK : e->fail(SG_EDEVICE, hipGetErrorString(err));
}

// The batched gravity launch on stream st (inputs prepared; stage timing
// is recorded on st through the first context).
sg_status ens_grav_launch(sg_ens* e, bool pot, hipStream_t st) {
    sg_ctx* c0 = e->c[0];
    hipStream_t own = c0->st;
    c0->st = st;
    c0->begin(SG_ST_GRAV);
    sg_launch_grav_ensemble(e->d_sys, e->d_tasks, e->ntasks, e->d_counter, pot ? 1 : 0, e->eps,
                            e->G, e->ipl, e->tile, e->nblocks, st);
    c0->end();
    c0->st = own;
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return e->fail(SG_EDEVICE, hipGetErrorString(err));
    for (sg_ctx* c : e->c) {
        c->have_grav = true;
        c->have_pot = pot;
    }
    return SG_OK;
}

sg_status ens_gravity(sg_ens* e, bool pot) {
    sg_status r = ens_grav_prep(e);
    return r != SG_OK ? r : ens_grav_launch(e, pot, e->st);
}

// Segmented update launches (all systems) with the contexts' bookkeeping.
sg_status ens_launched(sg_ens* e, const char* what) {
    hipError_t err = hipGetLastError();
    if (err == hipSuccess) return SG_OK;
    char m[256];
    snprintf(m, sizeof(m), "%s: %s", what, hipGetErrorString(err));
    return e->fail(SG_EDEVICE, m);
}

// Neighbour lists and density of every system that lacks them: one launch
// per stage for all systems when all lack them (every corrector), else
// system by system.
sg_status ens_lists_density(sg_ens* e) {
    sg_ctx* c0 = e->c[0];
    bool all_nbr = true, all_rho = true, any = false;
    for (sg_ctx* c : e->c) {
        all_nbr = all_nbr && !c->have_nbr;
        all_rho = all_rho && !c->have_rho;
        any = any || !c->have_nbr || !c->have_rho;
    }
    if (!any) return SG_OK;
    if (all_nbr && all_rho) {
        c0->begin(SG_ST_SORT);
        sg_seg_launch_sort(e->seg, e->st);
        c0->end();
        c0->begin(SG_ST_NBR);
        sg_seg_launch_nbr_search(e->seg, e->st);
        sg_seg_launch_scan_nbr(e->seg, e->st);
        sg_seg_launch_nbr_finish(e->seg, e->st);
        c0->end();
        c0->begin(SG_ST_DENSITY);
        sg_seg_launch_density(e->seg, e->st);
        c0->end();
        for (sg_ctx* c : e->c) {
            c->have_nbr = true;
            c->have_rho = true;
        }
        return ens_launched(e, "neighbour lists and density");
    }
    sg_status r;
    for (sg_ctx* c : e->c) {
        r = !c->have_nbr ? do_build(c) : SG_OK;
        if (r == SG_OK && !c->have_rho) r = do_density(c);
        if (r != SG_OK) return e->fail(r, c->msg);
    }
    return SG_OK;
}

sg_status ens_step(sg_ens* e, double dt, uint32_t flags) {
    if (flags & ~SG_POT) return e->fail(SG_EINVAL, "steps accept only SG_POT");
    if (!__builtin_isfinite(dt)) return e->fail(SG_EINVAL, "dt must be finite");
    const bool pot = (flags & SG_POT) != 0;
    sg_ctx* c0 = e->c[0];
    sg_status r;
    bool need_grav = false;
    // forces at r(t): lists and density are reused from the previous
    // corrector, gravity likewise (the first step computes them)
    for (sg_ctx* c : e->c) {
        if (c->predicted) return e->fail(SG_ESTATE, "step inside a predict/correct pair");
        need_grav |= !c->have_grav || (pot && !c->have_pot);
    }
    if ((r = ens_lists_density(e)) != SG_OK) return r;
    if (need_grav && (r = ens_gravity(e, pot)) != SG_OK) return r;
    // predictor: SPH right-hand side, total acceleration, update and the
    // gravity inputs at the predicted positions, each one launch for all
    c0->begin(SG_ST_SPH);
    sg_seg_launch_sph_state(e->seg, 0, e->st);
    c0->end();
    c0->begin(SG_ST_UPDATE);
    sg_seg_launch_combine(e->seg, e->st);
    sg_seg_launch_predict(e->seg, dt, e->st);
    c0->end();
    if ((r = ens_launched(e, "predictor")) != SG_OK) return r;
    for (sg_ctx* c : e->c) {
        c->invalidate_positions();
        c->predicted = true;
        c->accel_after_predict = false;
    }
    if ((r = ens_grav_prep(e)) != SG_OK) return r;
    // corrector right-hand side: the batched gravity beside every system's
    // neighbour build, density and SPH forces (disjoint buffers; the
    // gravity kernel reads only the prepared inputs), or before them with
    // step_serial (of the first context)
    auto chains = [&]() {
        sg_status q = ens_lists_density(e);
        if (q != SG_OK) return q;
        c0->begin(SG_ST_SPH);
        sg_seg_launch_sph_state(e->seg, 1, e->st);
        c0->end();
        for (sg_ctx* c : e->c) c->have_sph = true;
        return ens_launched(e, "SPH forces");
    };
    if (c0->prm.step_serial || !e->cst) {
        if ((r = ens_grav_launch(e, pot, e->st)) != SG_OK) return r;
        if ((r = chains()) != SG_OK) return r;
    } else {
        // the gravity on the contexts' stream, the chains on the second one
        // (forked before the gravity launch, joined back after the chains)
        if (hipEventRecord(e->cev[0], e->st) != hipSuccess ||
            hipStreamWaitEvent(e->cst, e->cev[0], 0) != hipSuccess)
            return e->fail(SG_EDEVICE, "fork to the chain stream failed");
        r = ens_grav_launch(e, pot, e->st);
        hipStream_t own = e->st;
        for (sg_ctx* c : e->c) c->st = e->cst;
        e->st = e->cst;
        sg_status rc = r == SG_OK ? chains() : r;
        e->st = own;
        for (sg_ctx* c : e->c) c->st = own;
        // join (also after an error, so that a capture stays whole)
        if ((hipEventRecord(e->cev[1], e->cst) != hipSuccess ||
             hipStreamWaitEvent(e->st, e->cev[1], 0) != hipSuccess) && rc == SG_OK)
            rc = e->fail(SG_EDEVICE, "join of the chain stream failed");
        if (rc != SG_OK) return rc;
    }
    // corrector update, one launch each for all systems
    c0->begin(SG_ST_UPDATE);
    sg_seg_launch_combine(e->seg, e->st);
    sg_seg_launch_correct(e->seg, dt, e->st);
    c0->end();
    for (sg_ctx* c : e->c) {
        c->accel_after_predict = true;
        c->predicted = false;
        c->have_sph = false;       // the SPH part was evaluated with the predicted velocities
    }
    return ens_launched(e, "corrector");
}

}  // namespace
}  // extern "C++"

size_t sg_ensemble_bytes(int32_t nsys, int64_t total_particles) {
    if (nsys < 1 || total_particles < 1) return 0;
    return ens_layout(nsys, total_particles / 64 + nsys).total;
}

sg_status sg_ensemble_create(sg_ctx* const* ctxs, int32_t nsys, void* d_ws, size_t ws_bytes,
                             void* chain_stream, sg_ens** out) {
    if (!out || !ctxs || nsys < 1) return SG_EINVAL;
    *out = nullptr;
    if (!d_ws || ((uintptr_t)d_ws & (kAlign - 1))) return SG_EINVAL;
    if (!ctxs[0] || !ctxs[0]->bound) return SG_EINVAL;
    if (chain_stream && chain_stream == (void*)ctxs[0]->st) return SG_EINVAL;
    std::vector<sg_ens_sys> sys((size_t)nsys);
    std::vector<sg_seg_sys> seg((size_t)nsys);
    std::vector<int64_t> pfx((size_t)SG_SEG_NPFX * (nsys + 1), 0);
    std::vector<std::pair<int64_t, sg_ens_task>> tasks;
    int64_t total = 0;
    int gas_passes = 1;
    // launch shape of the first context: 256 * ipl targets per task.  Unset
    // fields take the batched launch's measured best at 64 systems of
    // 8192-262144 particles, 2 targets per lane and 512 sources per tile
    // (the tasks fill the GPU whatever the systems' sizes, so the choice
    // does not follow the single-system rule).
    const int ipl = ctxs[0]->prm.grav_ipl != 0 ? ctxs[0]->prm.grav_ipl : 2;
    const int tile = ctxs[0]->prm.grav_tile != 0 ? ctxs[0]->prm.grav_tile : 512;
    const int64_t per = 256 * (int64_t)ipl;
    for (int32_t k = 0; k < nsys; ++k) {
        sg_ctx* c = ctxs[k];
        if (!c || !c->bound) return SG_EINVAL;
        if (c->prm.precision != SG_FP32C) return SG_EINVAL;
        if (c->st != ctxs[0]->st || c->prm.G != ctxs[0]->prm.G || c->prm.eps != ctxs[0]->prm.eps ||
            c->prm.grav_reorder != ctxs[0]->prm.grav_reorder)
            return SG_EINVAL;
        for (int32_t j = 0; j < k; ++j)
            if (ctxs[j] == c) return SG_EINVAL;      // each system once
        sg_ens_sys& S = sys[(size_t)k];
        sg_grav_sorted_ptrs(c->at<void>(c->L.gsorted), c->n, &S.xs, &S.ys, &S.zs, &S.ms, &S.sbox);
        S.order = c->at<int32_t>(c->L.gorder);
        S.n = c->n;
        S.gx = c->at<double>(c->L.gx);
        S.gy = c->at<double>(c->L.gy);
        S.gz = c->at<double>(c->L.gz);
        S.gp = c->s.pot ? c->s.pot : c->at<double>(c->L.gpot);
        const int64_t nb = (c->n + per - 1) / per;
        for (int64_t b = 0; b < nb; ++b) tasks.push_back({c->n, sg_ens_task{k, (int32_t)b}});
        total += c->n;
        // the segmented launches' view of the same system
        sg_seg_sys& Q = seg[(size_t)k];
        Q.x = c->s.x;
        Q.y = c->s.y;
        Q.z = c->s.z;
        Q.vx = c->s.vx;
        Q.vy = c->s.vy;
        Q.vz = c->s.vz;
        Q.m = c->s.m;
        Q.e = c->s.e;
        Q.ax = c->s.ax;
        Q.ay = c->s.ay;
        Q.az = c->s.az;
        Q.dedt = c->s.dedt;
        Q.rho = c->s.rho;
        Q.h = c->s.h;
        Q.key = c->at<int32_t>(c->L.key);
        Q.count = c->at<int32_t>(c->L.count);
        sg_morton_ptrs(c->at<void>(c->L.gsort), c->ng, &Q.gk0, &Q.gk1, &Q.gv0, &Q.gv1, &Q.ghist,
                       &Q.goffs, &Q.gntiles);
        Q.ncnt = c->at<int32_t>(c->L.ncnt);
        Q.slots = c->at<int32_t>(c->L.nbr_slots);
        Q.hmax = c->at<unsigned long long>(c->L.hmax);
        Q.off = c->at<int64_t>(c->L.off);
        Q.scan = c->at<void>(c->L.scan);
        Q.cell_cap = c->caps.cell_cap;
        Q.nnz_cap = c->caps.nnz_cap;
        Q.cell_scale = c->prm.cell_scale_log2 < 0 ? 0.5 : (c->prm.cell_scale_log2 > 0 ? 2.0 : 1.0);
        Q.vtx = c->at<double>(c->L.vtx);
        Q.vty = c->at<double>(c->L.vty);
        Q.vtz = c->at<double>(c->L.vtz);
        Q.et = c->at<double>(c->L.et);
        Q.asx = c->at<double>(c->L.asx);
        Q.asy = c->at<double>(c->L.asy);
        Q.asz = c->at<double>(c->L.asz);
        Q.gx = S.gx;
        Q.gy = S.gy;
        Q.gz = S.gz;
        Q.sph = c->sph();
        Q.g = c->grid();
        sg_morton_ptrs(c->at<void>(c->L.morton), c->n, &Q.mk0, &Q.mk1, &Q.mv0, &Q.mv1, &Q.mhist,
                       &Q.moffs, &Q.ntiles);
        Q.order = c->at<int32_t>(c->L.gorder);
        Q.xs = const_cast<double*>(S.xs);
        Q.ys = const_cast<double*>(S.ys);
        Q.zs = const_cast<double*>(S.zs);
        Q.ms = const_cast<double*>(S.ms);
        Q.sbox = const_cast<void*>(S.sbox);
        Q.n = c->n;
        Q.ng = c->ng;
        Q.gamma = c->prm.gamma;
        Q.alpha = c->prm.alpha;
        Q.beta = c->prm.beta;
        Q.eta = c->prm.eta;
        const bool gas = c->ng > 0;
        const int64_t cnt[SG_SEG_NPFX] = {(c->n + 255) / 256,
                                          (c->ng + 255) / 256,
                                          Q.ntiles,
                                          gas ? sg_cells_clear_blocks(c->caps.cell_cap) : 0,
                                          gas ? sg_scan_tiles(c->caps.cell_cap) : 0,
                                          gas ? sg_scan_tiles(c->ng) : 0,
                                          sg_compact_blocks(c->ng),
                                          gas ? Q.gntiles : 0,
                                          sg_sph_blocks(c->ng),
                                          sg_nbr_blocks(c->ng)};
        if (gas && sg_gas_radix_passes(c->caps.cell_cap) > gas_passes)
            gas_passes = sg_gas_radix_passes(c->caps.cell_cap);
        for (int q = 0; q < SG_SEG_NPFX; ++q)
            pfx[(size_t)q * (nsys + 1) + k + 1] = pfx[(size_t)q * (nsys + 1) + k] + cnt[q];
    }
    // largest systems first (their tasks are the longest)
    std::stable_sort(tasks.begin(), tasks.end(),
                     [](const std::pair<int64_t, sg_ens_task>& a,
                        const std::pair<int64_t, sg_ens_task>& b) { return a.first > b.first; });
    const ens_offsets o = ens_layout(nsys, (int64_t)tasks.size());
    if (ws_bytes < o.total || (int64_t)tasks.size() > total / 64 + nsys) return SG_EINVAL;
    std::vector<sg_ens_task> tk(tasks.size());
    for (size_t i = 0; i < tasks.size(); ++i) tk[i] = tasks[i].second;
    sg_ens* e = new (std::nothrow) sg_ens();
    if (!e) return SG_EINVAL;
    e->c.assign(ctxs, ctxs + nsys);
    e->st = ctxs[0]->st;
    char* ws = (char*)d_ws;
    e->d_sys = (sg_ens_sys*)ws;
    e->d_tasks = (sg_ens_task*)(ws + o.tasks);
    e->d_counter = (int32_t*)(ws + o.counter);
    e->ntasks = (int32_t)tk.size();
    e->ipl = ipl;
    e->tile = tile;
    e->eps = ctxs[0]->prm.eps;
    e->G = ctxs[0]->prm.G;
    e->seg.sys = (const sg_seg_sys*)(ws + o.seg);
    e->seg.pfx = (const int64_t*)(ws + o.pfx);
    e->seg.nsys = nsys;
    e->seg.gas_passes = gas_passes;
    for (int q = 0; q < SG_SEG_NPFX; ++q) e->seg.nblk[q] = pfx[(size_t)q * (nsys + 1) + nsys];
    e->msg[0] = 0;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // the chain stream: the caller's, else one with every CU in its mask.
    // A stream of the runtime's default kind shares one of the process's
    // few hardware queues with other streams, and a queue runs its packets
    // in order, so chains enqueued behind the persistent gravity kernel in a
    // shared queue would wait for it; a CU-masked stream gets a hardware
    // queue of its own.
    e->own_cst = chain_stream == nullptr;
    if (chain_stream) {
        e->cst = (hipStream_t)chain_stream;
    } else {
        std::vector<uint32_t> mask((size_t)((cus > 0 ? cus : 256) + 31) / 32, 0xffffffffu);
        if (cus > 0 && cus % 32) mask.back() = (1u << (cus % 32)) - 1u;
        if (hipExtStreamCreateWithCUMask(&e->cst, (uint32_t)mask.size(), mask.data()) != hipSuccess)
            e->cst = nullptr;
    }
    if (!e->cst || hipEventCreateWithFlags(&e->cev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&e->cev[1], hipEventDisableTiming) != hipSuccess) {
        if (e->cst && e->own_cst) (void)hipStreamDestroy(e->cst);   // fall back: one stream
        e->cst = nullptr;
        for (hipEvent_t& x : e->cev) {
            if (x) (void)hipEventDestroy(x);
            x = nullptr;
        }
    }
    // persistent grid: as many workgroups as are resident at once
    const int per_cu = sg_grav_ensemble_blocks_per_cu(ipl, tile, 1);
    (void)hipGetLastError();
    e->nblocks = per_cu * (cus > 0 ? cus : 256);
    if (e->nblocks > e->ntasks) e->nblocks = e->ntasks;
    if (hipMemcpyAsync(e->d_sys, sys.data(), sizeof(sg_ens_sys) * sys.size(), hipMemcpyHostToDevice,
                       e->st) != hipSuccess ||
        hipMemcpyAsync(e->d_tasks, tk.data(), sizeof(sg_ens_task) * tk.size(),
                       hipMemcpyHostToDevice, e->st) != hipSuccess ||
        hipMemcpyAsync(ws + o.seg, seg.data(), sizeof(sg_seg_sys) * seg.size(),
                       hipMemcpyHostToDevice, e->st) != hipSuccess ||
        hipMemcpyAsync(ws + o.pfx, pfx.data(), sizeof(int64_t) * pfx.size(), hipMemcpyHostToDevice,
                       e->st) != hipSuccess ||
        hipStreamSynchronize(e->st) != hipSuccess) {
        delete e;
        return SG_EDEVICE;
    }
    *out = e;
    return SG_OK;
}

sg_status sg_ensemble_gravity(sg_ens* e, uint32_t flags) {
    if (!e) return SG_EINVAL;
    if (flags & ~(SG_GRAV | SG_POT)) return e->fail(SG_EINVAL, "flags: SG_GRAV [| SG_POT]");
    (void)hipGetLastError();
    for (sg_ctx* c : e->c)
        if (c->predicted) return e->fail(SG_ESTATE, "gravity inside a predict/correct pair");
    sg_status r = ens_gravity(e, (flags & SG_POT) != 0);
    if (r != SG_OK) return r;
    for (sg_ctx* c : e->c) do_combine(c);
    return ens_launched(e, "combine");
}

sg_status sg_ensemble_step(sg_ens* e, double dt, uint32_t flags) {
    if (!e) return SG_EINVAL;
    (void)hipGetLastError();
    return ens_step(e, dt, flags);
}

sg_status sg_ensemble_run(sg_ens* e, double dt, int64_t nsteps, uint32_t flags, int32_t use_graph) {
    if (!e) return SG_EINVAL;
    if (nsteps < 0) return e->fail(SG_EINVAL, "nsteps must be >= 0");
    for (sg_ctx* c : e->c)
        if (use_graph && c->prof) return e->fail(SG_ESTATE, "stage timing must be off to capture");
    if (use_graph && nsteps >= 2 && e->st == nullptr)
        return e->fail(SG_EINVAL, "graph capture needs a stream other than the null stream");
    (void)hipGetLastError();
    // one period of the (common) Morton-order schedule per captured chunk
    const int64_t P = reorder_period(e->c[0]);
    const int64_t chunks = nsteps >= 1 ? (nsteps - 1) / P : 0;
    sg_status r;
    int64_t k = 0;
    if (!use_graph || chunks < 1) {
        for (; k < nsteps; ++k)
            if ((r = ens_step(e, dt, flags)) != SG_OK) return r;
        return hipStreamSynchronize(e->st) == hipSuccess ? SG_OK
                                                          : e->fail(SG_EDEVICE, "stream sync failed");
    }
    if ((r = ens_step(e, dt, flags)) != SG_OK) return r;
    ++k;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (hipStreamBeginCapture(e->st, hipStreamCaptureModeRelaxed) != hipSuccess)
        return e->fail(SG_EDEVICE, "hipStreamBeginCapture failed");
    sg_status rc = SG_OK;
    for (int64_t j = 0; j < P && rc == SG_OK; ++j) rc = ens_step(e, dt, flags);
    hipError_t ec = hipStreamEndCapture(e->st, &graph);
    if (rc != SG_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (ec != hipSuccess || !graph) return e->fail(SG_EDEVICE, "hipStreamEndCapture failed");
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return e->fail(SG_EDEVICE, "hipGraphInstantiate failed");
    }
    for (int64_t q = 0; q < chunks && rc == SG_OK; ++q, k += P)
        if (hipGraphLaunch(exec, e->st) != hipSuccess) rc = e->fail(SG_EDEVICE, "hipGraphLaunch failed");
    for (; k < nsteps && rc == SG_OK; ++k) rc = ens_step(e, dt, flags);
    if (hipStreamSynchronize(e->st) != hipSuccess && rc == SG_OK)
        rc = e->fail(SG_EDEVICE, "stream sync failed");
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return rc;
}

const char* sg_ensemble_last_error(const sg_ens* e) { return e ? e->msg : "null ensemble"; }

void sg_ensemble_destroy(sg_ens* e) { delete e; }

const char* sg_last_error(const sg_ctx* c) { return c ? c->msg : g_create_msg; }

sg_status sg_profile_enable(sg_ctx* c, int32_t on) {
    if (!c) return SG_EINVAL;
    (void)hipGetLastError();
    if (hipStreamSynchronize(c->st) != hipSuccess) return c->fail(SG_EDEVICE, "stream sync failed");
    for (auto& mk : c->marks) {
        c->pool.push_back(mk.a);
        c->pool.push_back(mk.b);
    }
    c->marks.clear();
    for (int k = 0; k < SG_NSTAGE; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_n[k] = 0;
    }
    c->prof = on != 0;
    return SG_OK;
}

sg_status sg_profile_read(sg_ctx* c, double ms[SG_NSTAGE], int64_t count[SG_NSTAGE]) {
    if (!c || !ms || !count) return SG_EINVAL;
    if (hipStreamSynchronize(c->st) != hipSuccess) return c->fail(SG_EDEVICE, "stream sync failed");
    for (auto& mk : c->marks) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, mk.a, mk.b) == hipSuccess) {
            c->prof_ms[mk.stage] += t;
            c->prof_n[mk.stage] += 1;
        }
        c->pool.push_back(mk.a);
        c->pool.push_back(mk.b);
    }
    c->marks.clear();
    for (int k = 0; k < SG_NSTAGE; ++k) {
        ms[k] = c->prof_ms[k];
        count[k] = c->prof_n[k];
    }
    return SG_OK;
}

void sg_destroy(sg_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->st);
    if (c->st2) {
        (void)hipStreamSynchronize(c->st2);
        (void)hipEventDestroy(c->ev_fork);
        (void)hipEventDestroy(c->ev_join);
    }
    for (auto& mk : c->marks) {
        (void)hipEventDestroy(mk.a);
        (void)hipEventDestroy(mk.b);
    }
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    if (c->is_static) {               // the slot and the array stay for the next one
        c->marks.clear();
        c->pool.clear();
        c->bound = false;
        static_release(c->dev);
        return;
    }
    delete c;
}

const char* sg_version(void) { return "sphgrav 0.1 gfx950"; }

}  // extern "C"

// sg_grav.hip -- direct (Particle-Particle) softened gravity, the paper's GFC
// kernel (Eq. self-gravity; O(N^2), Sec. 3), read with Plummer softening:
//   g_i = G sum_{j != i} m_j (r_j - r_i) / (|r_ij|^2 + eps^2)^{3/2},
//   phi_i = -G sum_{j != i} m_j / sqrt(|r_ij|^2 + eps^2).
//
// Tiling for CDNA4: a workgroup of 256 lanes owns 256*IPL targets held in
// registers; sources stream through LDS in tiles of 256 (double-buffered,
// one barrier per tile), every lane reading the same source (LDS
// broadcast).  The self pair is not skipped: it adds exactly 0 to g (zero
// separation) and m_i/eps to the potential sum, which is subtracted at the
// end.  A source range may be split across workgroups (grid.y) to fill the
// chip at small N; split partial sums are reduced in a fixed order.
//
// FP64 form: 1/sqrt by the hardware reciprocal square root refined with one
// third-order (Householder) step, y <- y (1 + e/2 + 3e^2/8), e = 1 - r2 y^2,
// which leaves FP64 rounding-level error for any starting error below 2^-17.
//
// FP32C form: each workgroup takes the position of its first target as an
// FP64 anchor P and works on FP32 offsets (float)(r - P), computed in FP64
// and rounded once, for targets and for every source tile.  Targets are in
// Morton order, so a workgroup's targets lie close to P and pair
// separations keep nearly full FP32 relative precision.  Pair arithmetic is
// FP32; each tile's partial sum is folded into a Kahan-compensated FP32
// accumulator; results are returned in FP64.
#include "sg_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kTile = 256;

struct alignas(16) d4 {
    double x, y, z, w;
};

// SEED32: start from the FP32 reciprocal square root of (float)r2 (relative
// error below 2^-23, on the transcendental pipe, which runs beside the main
// vector ALU) instead of the FP64 one (below 2^-24, a quarter-rate slot on
// the main ALU); r2 must then lie in the normal FP32 range (r2 >= eps^2).
template <bool SEED32>
__device__ inline double rsqrt_f64(double r2) {
    const double y0 = SEED32 ? (double)__builtin_amdgcn_rsqf((float)r2) : __builtin_amdgcn_rsq(r2);
    const double t = r2 * y0;
    const double e = __builtin_fma(-t, y0, 1.0);
    const double p = __builtin_fma(e, 0.375, 0.5);
    const double u = y0 * e;
    return __builtin_fma(u, p, y0);
}

template <int IPL, bool POT, bool SEED32>
__global__ __launch_bounds__(kBlock) void k_grav_f64(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ m, int64_t n, int64_t jchunk, double eps2, double G,
    double inv_eps, int final_out, double* __restrict__ ox, double* __restrict__ oy,
    double* __restrict__ oz, double* __restrict__ op, int64_t ostride) {
    __shared__ d4 tile[2][kTile];
    const int tid = threadIdx.x;
    const int64_t ib = (int64_t)blockIdx.x * (kBlock * IPL);
    double xi[IPL], yi[IPL], zi[IPL], ax[IPL], ay[IPL], az[IPL], ap[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int64_t i = ib + k * kBlock + tid;
        const bool v = i < n;
        xi[k] = v ? x[i] : 0.0;
        yi[k] = v ? y[i] : 0.0;
        zi[k] = v ? z[i] : 0.0;
        ax[k] = ay[k] = az[k] = ap[k] = 0.0;
    }
    const int64_t j0 = (int64_t)blockIdx.y * jchunk;
    int64_t j1 = j0 + jchunk;
    if (j1 > n) j1 = n;
    {
        const int64_t j = j0 + tid;
        d4 q{0, 0, 0, 0};
        if (j < j1) q = d4{x[j], y[j], z[j], m[j]};
        tile[0][tid] = q;
    }
    __syncthreads();
    int cur = 0;
    for (int64_t jt = j0; jt < j1; jt += kTile) {
        const bool more = jt + kTile < j1;
        d4 nq{0, 0, 0, 0};
        if (more) {
            const int64_t j = jt + kTile + tid;
            if (j < j1) nq = d4{x[j], y[j], z[j], m[j]};
        }
#pragma unroll 4
        for (int jj = 0; jj < kTile; ++jj) {
            const d4 q = tile[cur][jj];
#pragma unroll
            for (int k = 0; k < IPL; ++k) {
                const double dx = q.x - xi[k], dy = q.y - yi[k], dz = q.z - zi[k];
                const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
                const double rinv = rsqrt_f64<SEED32>(r2);
                const double mr = q.w * rinv;
                const double s = mr * (rinv * rinv);
                ax[k] = __builtin_fma(s, dx, ax[k]);
                ay[k] = __builtin_fma(s, dy, ay[k]);
                az[k] = __builtin_fma(s, dz, az[k]);
                if (POT) ap[k] += mr;
            }
        }
        if (more) tile[cur ^ 1][tid] = nq;
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int64_t i = ib + k * kBlock + tid;
        if (i >= n) continue;
        if (final_out) {
            ox[i] = G * ax[k];
            oy[i] = G * ay[k];
            oz[i] = G * az[k];
            if (POT) op[i] = -G * (ap[k] - m[i] * inv_eps);
        } else {
            const int64_t o = (int64_t)blockIdx.y * ostride + i;
            ox[o] = ax[k];
            oy[o] = ay[k];
            oz[o] = az[k];
            if (POT) op[o] = ap[k];
        }
    }
}

struct kahan {
    float s, c;
    __device__ inline void add(float v) {
        const float yv = v - c;
        const float t = s + yv;
        c = (t - s) - yv;
        s = t;
    }
    __device__ inline double value() const { return (double)s - (double)c; }
};

constexpr int kSub = 64;                 // sources per bounding box
constexpr double kNearFrac = 0.125;      // near field: box distance < D/8

// Box of a run of sorted positions: lo[3], hi[3].
struct box6 {
    double lo[3], hi[3];
};

__device__ inline double box_gap2(const box6& a, const box6& b) {
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
        double g = a.lo[d] - b.hi[d];
        const double g2 = b.lo[d] - a.hi[d];
        g = g > g2 ? g : g2;
        if (g > 0.0) s += g * g;
    }
    return s;
}

// FP32C form.  Sources and targets are both in Morton order (sorted FP64
// copies); each run of kSub sorted sources has a bounding box.  A workgroup
// anchors its targets at the centre P of their bounding box (diagonal D).
// Source sub-tiles whose box lies within D/8 of the target box (the near
// field) are evaluated with double-float offsets, (hi_j - hi_i) +
// (lo_j - lo_i) where hi = (float)(r - P) and lo = (float)((r - P) - hi), so
// close pairs keep full FP32 relative accuracy; all other sub-tiles use the
// single-float offsets hi_j - hi_i, whose rounding error is then at most a
// few units of 2^-24 of the pair separation.  The choice is uniform across
// the workgroup.
template <int IPL, bool POT>
__global__ __launch_bounds__(kBlock) void k_grav_f32c(
    const double* __restrict__ xs, const double* __restrict__ ys, const double* __restrict__ zs,
    const double* __restrict__ ms, const box6* __restrict__ sbox, const int32_t* __restrict__ order,
    int64_t n, int64_t jchunk, float eps2, double G, double inv_eps, int final_out,
    double* __restrict__ ox, double* __restrict__ oy, double* __restrict__ oz,
    double* __restrict__ op, int64_t ostride) {
    __shared__ float4 thi[2][kTile];
    __shared__ float4 tlo[2][kTile];
    __shared__ int s_near[2][kTile / kSub];
    const int tid = threadIdx.x;
    const int64_t ib = (int64_t)blockIdx.x * (kBlock * IPL);
    // bounding box of this workgroup's targets from the sub-tile boxes
    box6 bb;
    {
        const int64_t s0 = ib / kSub;
        int64_t s1 = (ib + kBlock * IPL + kSub - 1) / kSub;
        const int64_t nsub = (n + kSub - 1) / kSub;
        if (s1 > nsub) s1 = nsub;
        bb = sbox[s0];
        for (int64_t q = s0 + 1; q < s1; ++q) {
            const box6 o = sbox[q];
            for (int d = 0; d < 3; ++d) {
                bb.lo[d] = o.lo[d] < bb.lo[d] ? o.lo[d] : bb.lo[d];
                bb.hi[d] = o.hi[d] > bb.hi[d] ? o.hi[d] : bb.hi[d];
            }
        }
    }
    const double Px = 0.5 * (bb.lo[0] + bb.hi[0]);
    const double Py = 0.5 * (bb.lo[1] + bb.hi[1]);
    const double Pz = 0.5 * (bb.lo[2] + bb.hi[2]);
    double diag2 = 0.0;
    for (int d = 0; d < 3; ++d) diag2 += (bb.hi[d] - bb.lo[d]) * (bb.hi[d] - bb.lo[d]);
    const double near2 = kNearFrac * kNearFrac * diag2;

    float xh[IPL], yh[IPL], zh[IPL], xl[IPL], yl[IPL], zl[IPL];
    float tx[IPL], ty[IPL], tz[IPL], tp[IPL];
    kahan sx[IPL], sy[IPL], sz[IPL], sp[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        int64_t i = ib + k * kBlock + tid;
        if (i >= n) i = ib;
        const double dx = xs[i] - Px, dy = ys[i] - Py, dz = zs[i] - Pz;
        xh[k] = (float)dx;
        yh[k] = (float)dy;
        zh[k] = (float)dz;
        xl[k] = (float)(dx - (double)xh[k]);
        yl[k] = (float)(dy - (double)yh[k]);
        zl[k] = (float)(dz - (double)zh[k]);
        sx[k] = sy[k] = sz[k] = sp[k] = kahan{0.0f, 0.0f};
    }
    const int64_t j0 = (int64_t)blockIdx.y * jchunk;
    int64_t j1 = j0 + jchunk;
    if (j1 > n) j1 = n;

    // stage one tile of sources (and the near flags of its sub-tiles)
    auto stage = [&](int buf, int64_t jt) {
        const int64_t j = jt + tid;
        float4 h = make_float4(0.f, 0.f, 0.f, 0.f), l = make_float4(0.f, 0.f, 0.f, 0.f);
        if (j < j1) {
            const double dx = xs[j] - Px, dy = ys[j] - Py, dz = zs[j] - Pz;
            h = make_float4((float)dx, (float)dy, (float)dz, (float)ms[j]);
            l = make_float4((float)(dx - (double)h.x), (float)(dy - (double)h.y),
                            (float)(dz - (double)h.z), 0.f);
        }
        thi[buf][tid] = h;
        tlo[buf][tid] = l;
        if (tid < kTile / kSub) {
            const int64_t q = jt / kSub + tid;
            int nr = 0;
            if (jt + (int64_t)tid * kSub < j1) nr = box_gap2(bb, sbox[q]) < near2;
            s_near[buf][tid] = nr;
        }
    };

    stage(0, j0);
    __syncthreads();
    int cur = 0;
    for (int64_t jt = j0; jt < j1; jt += kTile) {
        const bool more = jt + kTile < j1;
#pragma unroll
        for (int k = 0; k < IPL; ++k) tx[k] = ty[k] = tz[k] = tp[k] = 0.0f;
        for (int sb = 0; sb < kTile / kSub; ++sb) {
            if (s_near[cur][sb]) {
#pragma unroll 2
                for (int jj = sb * kSub; jj < (sb + 1) * kSub; ++jj) {
                    const float4 q = thi[cur][jj];
                    const float4 ql = tlo[cur][jj];
#pragma unroll
                    for (int k = 0; k < IPL; ++k) {
                        const float dx = (q.x - xh[k]) + (ql.x - xl[k]);
                        const float dy = (q.y - yh[k]) + (ql.y - yl[k]);
                        const float dz = (q.z - zh[k]) + (ql.z - zl[k]);
                        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2)));
                        const float rinv = __builtin_amdgcn_rsqf(r2);
                        const float mr = q.w * rinv;
                        const float s = mr * (rinv * rinv);
                        tx[k] = __builtin_fmaf(s, dx, tx[k]);
                        ty[k] = __builtin_fmaf(s, dy, ty[k]);
                        tz[k] = __builtin_fmaf(s, dz, tz[k]);
                        if (POT) tp[k] += mr;
                    }
                }
            } else {
#pragma unroll 4
                for (int jj = sb * kSub; jj < (sb + 1) * kSub; ++jj) {
                    const float4 q = thi[cur][jj];
#pragma unroll
                    for (int k = 0; k < IPL; ++k) {
                        const float dx = q.x - xh[k], dy = q.y - yh[k], dz = q.z - zh[k];
                        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2)));
                        const float rinv = __builtin_amdgcn_rsqf(r2);
                        const float mr = q.w * rinv;
                        const float s = mr * (rinv * rinv);
                        tx[k] = __builtin_fmaf(s, dx, tx[k]);
                        ty[k] = __builtin_fmaf(s, dy, ty[k]);
                        tz[k] = __builtin_fmaf(s, dz, tz[k]);
                        if (POT) tp[k] += mr;
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
            sx[k].add(tx[k]);
            sy[k].add(ty[k]);
            sz[k].add(tz[k]);
            if (POT) sp[k].add(tp[k]);
        }
        __syncthreads();                       // everyone is done with tile `cur`
        if (more) stage(cur ^ 1, jt + kTile);
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int64_t i = ib + k * kBlock + tid;
        if (i >= n) continue;
        int32_t t = order[i];
        if ((uint64_t)t >= (uint64_t)n) continue;
        if (final_out) {
            ox[t] = G * sx[k].value();
            oy[t] = G * sy[k].value();
            oz[t] = G * sz[k].value();
            if (POT) op[t] = -G * (sp[k].value() - ms[i] * inv_eps);
        } else {
            const int64_t o = (int64_t)blockIdx.y * ostride + t;
            ox[o] = sx[k].value();
            oy[o] = sy[k].value();
            oz[o] = sz[k].value();
            if (POT) op[o] = sp[k].value();
        }
    }
}

// FP32C form with the far field on the matrix cores.  For a far pair the
// squared separation expands as r^2 = (|x_i|^2 + eps^2) - 2 x_i . x_j
// + |x_j|^2, a rank-4 product: one v_mfma_f32_16x16x4f32 gives it for 16
// targets x 16 sources, with A[i] = (x_i, y_i, z_i, 1), B[j] = (-2x_j,
// -2y_j, -2z_j, |x_j|^2) and C[i] = |x_i|^2 + eps^2 (offsets from the
// anchor P, FP32).  The acceleration is accumulated as sum_j s_ij x_j -
// x_i sum_j s_ij.  Both rewritings lose accuracy only when |x_i|, |x_j| are
// large against |r_ij|; sources nearer than max(D/8, 4 eps) to the target
// box are therefore evaluated as in k_grav_f32c's near field (double-float
// offsets, one target per lane), and for the rest |x| <= 5|r|.  Per
// workgroup: 4 wavefronts of 16 targets; sources stream through LDS in
// tiles of kMT.  Lane l of the matrix product holds rows 4(l/16)..+3 and
// source column l%16.
constexpr int kMT = 512;
typedef float v4f __attribute__((ext_vector_type(4)));

struct f32m_lds {
    float4 hi[2][kMT];          // (x, y, z, m) hi parts, anchor-relative
    float4 lo[2][kMT];          // (x, y, z) lo parts
    float4 mx[2][kMT];          // (m x, m y, m z, m) for the far-field sums
    float b[2][4][kMT];         // B operand (-2x, -2y, -2z, |x|^2)
    int near[2][kMT / kSub];
    double out[kBlock / 64][16][9];
};

// One workgroup task: targets ib .. ib+63 (sorted order) against sources
// [j0, j1).  Outputs go to particle order (order[]) at ox[w + t] etc.,
// w = out_off; raw sums unless final_out.
template <bool POT>
__device__ __attribute__((always_inline)) inline void f32m_task(f32m_lds& L, const double* __restrict__ xs,
                          const double* __restrict__ ys, const double* __restrict__ zs,
                          const double* __restrict__ ms, const box6* __restrict__ sbox,
                          const int32_t* __restrict__ order, int64_t n, int64_t ib, int64_t j0,
                          int64_t j1, double eps, double G, int final_out,
                          double* __restrict__ ox, double* __restrict__ oy,
                          double* __restrict__ oz, double* __restrict__ op, int64_t out_off) {
    auto& s_hi = L.hi;
    auto& s_lo = L.lo;
    auto& s_b = L.b;
    auto& s_mx = L.mx;
    auto& s_near = L.near;
    auto& s_out = L.out;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int col = lane & 15, grp = lane >> 4;
    const box6 bb = sbox[ib / kSub];                           // box of the 64 targets
    const double Px = 0.5 * (bb.lo[0] + bb.hi[0]);
    const double Py = 0.5 * (bb.lo[1] + bb.hi[1]);
    const double Pz = 0.5 * (bb.lo[2] + bb.hi[2]);
    double diag2 = 0.0;
    for (int d = 0; d < 3; ++d) diag2 += (bb.hi[d] - bb.lo[d]) * (bb.hi[d] - bb.lo[d]);
    double near2 = kNearFrac * kNearFrac * diag2;
    near2 = near2 > 16.0 * eps * eps ? near2 : 16.0 * eps * eps;
    const float eps2f = (float)(eps * eps);

    // target of this lane for the A operand and the near field: t = col
    int64_t it = ib + wave * 16 + col;
    if (it >= n) it = ib;
    const double tdx = xs[it] - Px, tdy = ys[it] - Py, tdz = zs[it] - Pz;
    const float hx = (float)tdx, hy = (float)tdy, hz = (float)tdz;
    const float lx = (float)(tdx - (double)hx), ly = (float)(tdy - (double)hy),
                lz = (float)(tdz - (double)hz);
    const float a_op = grp == 0 ? hx : (grp == 1 ? hy : (grp == 2 ? hz : 1.0f));
    // C operand: rows 4*grp + r of this wave's 16 targets
    v4f cop;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        int64_t ic = ib + wave * 16 + 4 * grp + r;
        if (ic >= n) ic = ib;
        const double cx = xs[ic] - Px, cy = ys[ic] - Py, cz = zs[ic] - Pz;
        cop[r] = (float)(cx * cx + cy * cy + cz * cz + eps * eps);
    }
    float fx[4], fy[4], fz[4], f1[4], fp[4];
    double Fx[4], Fy[4], Fz[4], F1[4], Fp[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        fx[r] = fy[r] = fz[r] = f1[r] = fp[r] = 0.0f;
        Fx[r] = Fy[r] = Fz[r] = F1[r] = Fp[r] = 0.0;
    }
    float nx = 0.f, ny = 0.f, nz = 0.f, np = 0.f;
    double Nx = 0.0, Ny = 0.0, Nz = 0.0, Np = 0.0;

    auto stage = [&](int buf, int64_t jt) {
#pragma unroll
        for (int u = 0; u < kMT / kBlock; ++u) {
            const int jl = u * kBlock + tid;
            const int64_t j = jt + jl;
            float4 h = make_float4(0.f, 0.f, 0.f, 0.f), l = make_float4(0.f, 0.f, 0.f, 0.f);
            float q2 = 0.f;
            if (j < j1) {
                const double dx = xs[j] - Px, dy = ys[j] - Py, dz = zs[j] - Pz;
                h = make_float4((float)dx, (float)dy, (float)dz, (float)ms[j]);
                l = make_float4((float)(dx - (double)h.x), (float)(dy - (double)h.y),
                                (float)(dz - (double)h.z), 0.f);
                q2 = (float)(dx * dx + dy * dy + dz * dz);
            }
            s_hi[buf][jl] = h;
            s_lo[buf][jl] = l;
            s_mx[buf][jl] = make_float4(h.w * h.x, h.w * h.y, h.w * h.z, h.w);
            s_b[buf][0][jl] = -2.0f * h.x;
            s_b[buf][1][jl] = -2.0f * h.y;
            s_b[buf][2][jl] = -2.0f * h.z;
            s_b[buf][3][jl] = q2;
        }
        if (tid < kMT / kSub) {
            const int64_t q = jt / kSub + tid;
            int nr = 0;
            if (jt + (int64_t)tid * kSub < j1) nr = box_gap2(bb, sbox[q]) < near2;
            s_near[buf][tid] = nr;
        }
    };

    stage(0, j0);
    __syncthreads();
    int cur = 0;
    for (int64_t jt = j0; jt < j1; jt += kMT) {
        const bool more = jt + kMT < j1;
        for (int sb = 0; sb < kMT / kSub; ++sb) {
            if (s_near[cur][sb]) {
                // near field: target col, sources sb*64 + 4k + grp
#pragma unroll 4
                for (int k = 0; k < kSub / 4; ++k) {
                    const int jl = sb * kSub + 4 * k + grp;
                    const float4 q = s_hi[cur][jl];
                    const float4 ql = s_lo[cur][jl];
                    const float dx = (q.x - hx) + (ql.x - lx);
                    const float dy = (q.y - hy) + (ql.y - ly);
                    const float dz = (q.z - hz) + (ql.z - lz);
                    const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2f)));
                    const float rinv = __builtin_amdgcn_rsqf(r2);
                    const float mr = q.w * rinv;
                    const float sv = mr * (rinv * rinv);
                    nx = __builtin_fmaf(sv, dx, nx);
                    ny = __builtin_fmaf(sv, dy, ny);
                    nz = __builtin_fmaf(sv, dz, nz);
                    if (POT) np += mr;
                }
            } else {
#pragma unroll 2
                for (int c = 0; c < kSub / 16; ++c) {
                    const int jl = sb * kSub + c * 16 + col;
                    const float b = s_b[cur][grp][jl];
                    const v4f d = __builtin_amdgcn_mfma_f32_16x16x4f32(a_op, b, cop, 0, 0, 0);
                    const float4 q = s_mx[cur][jl];           // (m x, m y, m z, m) of source jl
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float rinv = __builtin_amdgcn_rsqf(d[r]);
                        const float rinv3 = (rinv * rinv) * rinv;
                        fx[r] = __builtin_fmaf(rinv3, q.x, fx[r]);
                        fy[r] = __builtin_fmaf(rinv3, q.y, fy[r]);
                        fz[r] = __builtin_fmaf(rinv3, q.z, fz[r]);
                        f1[r] = __builtin_fmaf(rinv3, q.w, f1[r]);
                        if (POT) fp[r] = __builtin_fmaf(rinv, q.w, fp[r]);
                    }
                }
            }
        }
        // fold this tile's FP32 partial sums into FP64
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Fx[r] += (double)fx[r];
            Fy[r] += (double)fy[r];
            Fz[r] += (double)fz[r];
            F1[r] += (double)f1[r];
            if (POT) Fp[r] += (double)fp[r];
            fx[r] = fy[r] = fz[r] = f1[r] = fp[r] = 0.0f;
        }
        Nx += (double)nx;
        Ny += (double)ny;
        Nz += (double)nz;
        if (POT) Np += (double)np;
        nx = ny = nz = np = 0.0f;
        __syncthreads();
        if (more) stage(cur ^ 1, jt + kMT);
        __syncthreads();
        cur ^= 1;
    }
    // far sums: reduce over the 16 source columns of each row group
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        for (int o = 1; o < 16; o <<= 1) {
            Fx[r] += __shfl_xor(Fx[r], o, 64);
            Fy[r] += __shfl_xor(Fy[r], o, 64);
            Fz[r] += __shfl_xor(Fz[r], o, 64);
            F1[r] += __shfl_xor(F1[r], o, 64);
            if (POT) Fp[r] += __shfl_xor(Fp[r], o, 64);
        }
    }
    // near sums: reduce over the 4 source quarters of each target
    for (int o = 16; o < 64; o <<= 1) {
        Nx += __shfl_xor(Nx, o, 64);
        Ny += __shfl_xor(Ny, o, 64);
        Nz += __shfl_xor(Nz, o, 64);
        if (POT) Np += __shfl_xor(Np, o, 64);
    }
    if (col == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double* o = s_out[wave][4 * grp + r];
            o[0] = Fx[r];
            o[1] = Fy[r];
            o[2] = Fz[r];
            o[3] = F1[r];
            o[4] = Fp[r];
        }
    }
    if (grp == 0) {
        double* o = s_out[wave][col];
        o[5] = Nx;
        o[6] = Ny;
        o[7] = Nz;
        o[8] = Np;
    }
    __syncthreads();
    if (grp == 0) {
        const int64_t i = ib + wave * 16 + col;
        if (i < n) {
            int32_t t = order[i];
            if ((uint64_t)t < (uint64_t)n) {
                const double* o = s_out[wave][col];
                const double gx = o[0] - (double)hx * o[3] + o[5];
                const double gy = o[1] - (double)hy * o[3] + o[6];
                const double gz = o[2] - (double)hz * o[3] + o[7];
                const double pp = o[4] + o[8];
                if (final_out) {
                    ox[t] = G * gx;
                    oy[t] = G * gy;
                    oz[t] = G * gz;
                    if (POT) op[t] = -G * (pp - ms[i] / eps);
                } else {
                    const int64_t w = out_off + t;
                    ox[w] = gx;
                    oy[w] = gy;
                    oz[w] = gz;
                    if (POT) op[w] = pp;
                }
            }
        }
    }
    __syncthreads();                             // LDS free for the next task
}

template <bool POT>
__global__ __launch_bounds__(kBlock) void k_grav_f32m(
    const double* __restrict__ xs, const double* __restrict__ ys, const double* __restrict__ zs,
    const double* __restrict__ ms, const box6* __restrict__ sbox, const int32_t* __restrict__ order,
    int64_t n, int64_t jchunk, double eps, double G, int final_out, double* __restrict__ ox,
    double* __restrict__ oy, double* __restrict__ oz, double* __restrict__ op, int64_t ostride) {
    __shared__ f32m_lds L;
    const int64_t j0 = (int64_t)blockIdx.y * jchunk;
    int64_t j1 = j0 + jchunk;
    if (j1 > n) j1 = n;
    f32m_task<POT>(L, xs, ys, zs, ms, sbox, order, n, (int64_t)blockIdx.x * 64, j0, j1, eps, G,
                   final_out, ox, oy, oz, op, (int64_t)blockIdx.y * ostride);
}

// Persistent launch over the target blocks of several independent systems:
// each workgroup takes the next (system, block) task from a counter until
// none is left; tasks are listed largest system first.
template <bool POT>
__global__ __launch_bounds__(kBlock) void k_grav_f32m_ens(const sg_ens_sys* __restrict__ sys,
                                                          const sg_ens_task* __restrict__ tasks,
                                                          int32_t ntasks, int32_t* counter,
                                                          double eps, double G) {
    __shared__ f32m_lds L;
    __shared__ int32_t s_task;
    for (;;) {
        if (threadIdx.x == 0) s_task = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t t = s_task;
        __syncthreads();
        if (t >= ntasks) break;                  // uniform: every wavefront leaves here
        const sg_ens_task tk = tasks[t];
        const sg_ens_sys S = sys[tk.sys];
        f32m_task<POT>(L, S.xs, S.ys, S.zs, S.ms, (const box6*)S.sbox, S.order, S.n,
                       (int64_t)tk.blk * 64, 0, S.n, eps, G, 1, S.gx, S.gy, S.gz, S.gp, 0);
    }
}

__global__ void k_counter_reset(int32_t* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

// Gather positions and masses into Morton order and build the bounding box
// of every run of kSub sorted particles (one wavefront per run).
__global__ __launch_bounds__(kBlock) void k_sorted_boxes(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ m, const int32_t* __restrict__ order, int64_t n,
    double* __restrict__ xs, double* __restrict__ ys, double* __restrict__ zs,
    double* __restrict__ ms, box6* __restrict__ sbox) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool v = i < n;
    double p[3] = {0, 0, 0};
    if (v) {
        int32_t t = order[i];
        if ((uint64_t)t >= (uint64_t)n) t = 0;
        p[0] = x[t];
        p[1] = y[t];
        p[2] = z[t];
        xs[i] = p[0];
        ys[i] = p[1];
        zs[i] = p[2];
        ms[i] = m[t];
    }
    box6 b;
    for (int d = 0; d < 3; ++d) {
        double lo = v ? p[d] : __builtin_inf(), hi = v ? p[d] : -__builtin_inf();
        for (int o = 32; o > 0; o >>= 1) {
            const double a = __shfl_xor(lo, o, 64), c = __shfl_xor(hi, o, 64);
            lo = a < lo ? a : lo;
            hi = c > hi ? c : hi;
        }
        b.lo[d] = lo;
        b.hi[d] = hi;
    }
    const int64_t q = i / kSub;
    if ((threadIdx.x & 63) == 0 && q * kSub < n) sbox[q] = b;
}

__global__ __launch_bounds__(kBlock) void k_grav_reduce(const double* __restrict__ part,
                                                        const double* __restrict__ m, int64_t n,
                                                        int split, int with_pot, double G,
                                                        double inv_eps, double* __restrict__ gx,
                                                        double* __restrict__ gy,
                                                        double* __restrict__ gz,
                                                        double* __restrict__ gp) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t stride = (int64_t)split * n;     // component stride
    double sx = 0, sy = 0, sz = 0, sp = 0;
    for (int s = 0; s < split; ++s) {
        const int64_t o = (int64_t)s * n + i;
        sx += part[o];
        sy += part[stride + o];
        sz += part[2 * stride + o];
        if (with_pot) sp += part[3 * stride + o];
    }
    gx[i] = G * sx;
    gy[i] = G * sy;
    gz[i] = G * sz;
    if (with_pot) gp[i] = -G * (sp - m[i] * inv_eps);
}

template <int IPL, bool POT>
void launch_t(const sg_grav_args& a, dim3 grid, int64_t jchunk, int final_out, double* ox,
              double* oy, double* oz, double* op, int64_t ostride, hipStream_t st) {
    const double inv_eps = 1.0 / a.eps;
    if (a.precision == SG_FP32C)
        hipLaunchKernelGGL((k_grav_f32c<IPL, POT>), grid, dim3(kBlock), 0, st, a.xs, a.ys, a.zs,
                           a.ms, (const box6*)a.sbox, a.order, a.n, jchunk,
                           (float)(a.eps * a.eps), a.G, inv_eps, final_out, ox, oy, oz, op,
                           ostride);
    else if (a.variant == 2)
        hipLaunchKernelGGL((k_grav_f64<IPL, POT, false>), grid, dim3(kBlock), 0, st, a.x, a.y, a.z,
                           a.m, a.n, jchunk, a.eps * a.eps, a.G, inv_eps, final_out, ox, oy, oz,
                           op, ostride);
    else
        hipLaunchKernelGGL((k_grav_f64<IPL, POT, true>), grid, dim3(kBlock), 0, st, a.x, a.y, a.z,
                           a.m, a.n, jchunk, a.eps * a.eps, a.G, inv_eps, final_out, ox, oy, oz,
                           op, ostride);
}

template <int IPL>
void launch_ipl(const sg_grav_args& a, dim3 grid, int64_t jchunk, int final_out, double* ox,
                double* oy, double* oz, double* op, int64_t ostride, hipStream_t st) {
    if (a.with_pot)
        launch_t<IPL, true>(a, grid, jchunk, final_out, ox, oy, oz, op, ostride, st);
    else
        launch_t<IPL, false>(a, grid, jchunk, final_out, ox, oy, oz, op, ostride, st);
}

}  // namespace

size_t sg_grav_sorted_bytes(int64_t n) {
    const int64_t nsub = (n + kSub - 1) / kSub;
    return 4 * ((8 * (size_t)n + 255) & ~(size_t)255) + sizeof(box6) * (size_t)nsub + 256;
}

namespace {
void sorted_views(sg_grav_args& a) {
    const size_t col = (8 * (size_t)a.n + 255) & ~(size_t)255;
    char* b = (char*)a.sorted;
    a.xs = (double*)b;
    a.ys = (double*)(b + col);
    a.zs = (double*)(b + 2 * col);
    a.ms = (double*)(b + 3 * col);
    a.sbox = b + 4 * col;
}
}  // namespace

void sg_grav_sorted_ptrs(void* sorted, int64_t n, const double** xs, const double** ys,
                         const double** zs, const double** ms, const void** sbox) {
    sg_grav_args a;
    a.sorted = sorted;
    a.n = n;
    sorted_views(a);
    *xs = a.xs;
    *ys = a.ys;
    *zs = a.zs;
    *ms = a.ms;
    *sbox = a.sbox;
}

void sg_launch_grav_ensemble(const sg_ens_sys* d_sys, const sg_ens_task* d_tasks, int32_t ntasks,
                             int32_t* d_counter, int with_pot, double eps, double G, int nblocks,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_counter_reset, dim3(1), dim3(64), 0, st, d_counter);
    if (with_pot)
        hipLaunchKernelGGL((k_grav_f32m_ens<true>), dim3(nblocks), dim3(kBlock), 0, st, d_sys,
                           d_tasks, ntasks, d_counter, eps, G);
    else
        hipLaunchKernelGGL((k_grav_f32m_ens<false>), dim3(nblocks), dim3(kBlock), 0, st, d_sys,
                           d_tasks, ntasks, d_counter, eps, G);
}

int sg_launch_grav_sorted(const sg_grav_args& a_in, hipStream_t st) {
    if (!a_in.order || !a_in.sorted || !a_in.x || !a_in.y || !a_in.z || !a_in.m || a_in.n < 1)
        return -1;
    sg_grav_args a = a_in;
    sorted_views(a);
    const unsigned nb = (unsigned)((a.n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_sorted_boxes, dim3(nb), dim3(kBlock), 0, st, a.x, a.y, a.z, a.m, a.order,
                       a.n, (double*)a.xs, (double*)a.ys, (double*)a.zs, (double*)a.ms,
                       (box6*)a.sbox);
    return 0;
}

int sg_launch_gravity(const sg_grav_args& a_in, hipStream_t st) {
    if (!a_in.x || !a_in.y || !a_in.z || !a_in.m || !a_in.gx || !a_in.gy || !a_in.gz ||
        !a_in.gpot || !a_in.part || a_in.n < 1)
        return -1;
    if (a_in.precision == SG_FP32C && (!a_in.order || !a_in.sorted)) return -1;
    sg_grav_args a = a_in;
    if (a.precision == SG_FP32C) sorted_views(a);
    const bool mfma = a.precision == SG_FP32C && a.variant == 2;
    const int ipl = a.ipl;
    const int64_t per = mfma ? 64 : (int64_t)kBlock * ipl;
    const int64_t iblocks = (a.n + per - 1) / per;
    int split = a.split < 1 ? 1 : a.split;
    // source chunk: a multiple of the tile, covering n in `split` pieces
    const int64_t tile = mfma ? kMT : kTile;
    int64_t jchunk = (a.n + split - 1) / split;
    jchunk = (jchunk + tile - 1) / tile * tile;
    split = (int)((a.n + jchunk - 1) / jchunk);
    const dim3 grid((unsigned)iblocks, (unsigned)split);
    const int final_out = split == 1;
    double *ox = a.gx, *oy = a.gy, *oz = a.gz, *op = a.gpot;
    const int64_t ostride = a.n;
    if (!final_out) {
        const int64_t comp = (int64_t)split * a.n;
        ox = a.part;
        oy = a.part + comp;
        oz = a.part + 2 * comp;
        op = a.part + 3 * comp;
    }
    if (mfma) {
        if (a.with_pot)
            hipLaunchKernelGGL((k_grav_f32m<true>), grid, dim3(kBlock), 0, st, a.xs, a.ys, a.zs, a.ms,
                               (const box6*)a.sbox, a.order, a.n, jchunk, a.eps, a.G, final_out,
                               ox, oy, oz, op, ostride);
        else
            hipLaunchKernelGGL((k_grav_f32m<false>), grid, dim3(kBlock), 0, st, a.xs, a.ys, a.zs,
                               a.ms, (const box6*)a.sbox, a.order, a.n, jchunk, a.eps, a.G,
                               final_out, ox, oy, oz, op, ostride);
    } else switch (ipl) {
        case 1: launch_ipl<1>(a, grid, jchunk, final_out, ox, oy, oz, op, ostride, st); break;
        case 2: launch_ipl<2>(a, grid, jchunk, final_out, ox, oy, oz, op, ostride, st); break;
        default: launch_ipl<4>(a, grid, jchunk, final_out, ox, oy, oz, op, ostride, st); break;
    }
    if (!final_out) {
        const unsigned nb = (unsigned)((a.n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_grav_reduce, dim3(nb), dim3(kBlock), 0, st, a.part, a.m, a.n, split,
                           a.with_pot, a.G, 1.0 / a.eps, a.gx, a.gy, a.gz, a.gpot);
    }
    return 0;
}

// sg_grav.hip -- direct (Particle-Particle) softened gravity, the paper's GFC
// kernel (Eq. self-gravity; O(N^2), Sec. 3), read with Plummer softening:
//   g_i = G sum_{j != i} m_j (r_j - r_i) / (|r_ij|^2 + eps^2)^{3/2},
//   phi_i = -G sum_{j != i} m_j / sqrt(|r_ij|^2 + eps^2).
//
// Tiling for CDNA4: a workgroup of 256 lanes owns 256*IPL targets held in
// registers; sources stream through LDS in tiles of TILE (128, 256 or 512;
// double-buffered, one barrier per tile), every lane reading the same
// source (LDS broadcast).  The self pair is not skipped: it adds exactly 0
// to g (zero separation) and m_i/eps to the potential sum, which is
// subtracted at the end.  A source range may be split across workgroups
// (grid.y) to fill the chip at small N; split partial sums are reduced in a
// fixed order.  All pair work is on the vector ALU: per pair the kernel is
// bound by instruction issue, not by memory (sources are re-read from L2 by
// every workgroup, a few GB/s of HBM traffic in all).
//
// FP64 form: 1/sqrt by the hardware reciprocal square root refined with one
// third-order (Householder) step, y <- y (1 + e/2 + 3e^2/8), e = 1 - r2 y^2,
// which leaves FP64 rounding-level error for any starting error below 2^-17.
//
// FP32C form: see k_grav_f32c below (Morton-ordered particles, FP64 anchor
// per workgroup, FP32 pair arithmetic, Kahan-compensated FP32 partial sums).
#include "sg_internal.h"

namespace {

constexpr int kBlock = 256;

struct alignas(16) d4 {
    double x, y, z, w;
};

// SEED32: start from the FP32 reciprocal square root of (float)r2 (relative
// error below 2^-23, on the transcendental pipe) instead of the FP64 one
// (below 2^-24, a quarter-rate slot on the main ALU); r2 must then lie in
// the normal FP32 range (r2 >= eps^2).
template <bool SEED32>
__device__ inline double rsqrt_f64(double r2) {
    const double y0 = SEED32 ? (double)__builtin_amdgcn_rsqf((float)r2) : __builtin_amdgcn_rsq(r2);
    const double t = r2 * y0;
    const double e = __builtin_fma(-t, y0, 1.0);
    const double p = __builtin_fma(e, 0.375, 0.5);
    const double u = y0 * e;
    return __builtin_fma(u, p, y0);
}

template <int IPL, int TILE, bool POT, bool SEED32>
__global__ __launch_bounds__(kBlock) void k_grav_f64(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ m, int64_t n, int64_t jchunk, double eps2, double G,
    double inv_eps, int final_out, double* __restrict__ ox, double* __restrict__ oy,
    double* __restrict__ oz, double* __restrict__ op, int64_t ostride) {
    constexpr int kPer = (TILE + kBlock - 1) / kBlock;   // sources staged per lane
    __shared__ d4 tile[2][TILE];
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
    // sources past j1 stage as massless points at the origin
    auto fetch = [&](int64_t jt, d4* q) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t j = jt + u * kBlock + tid;
            q[u] = d4{0, 0, 0, 0};
            if (j < j1) q[u] = d4{x[j], y[j], z[j], m[j]};
        }
    };
    auto put = [&](int buf, const d4* q) {
#pragma unroll
        for (int u = 0; u < kPer; ++u)
            if (u * kBlock + tid < TILE) tile[buf][u * kBlock + tid] = q[u];
    };
    d4 nq[kPer];
    fetch(j0, nq);
    put(0, nq);
    __syncthreads();
    int cur = 0;
    for (int64_t jt = j0; jt < j1; jt += TILE) {
        const bool more = jt + TILE < j1;
        if (more) fetch(jt + TILE, nq);
#pragma unroll 4
        for (int jj = 0; jj < TILE; ++jj) {
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
        if (more) put(cur ^ 1, nq);
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
// anchors its targets at the centre P of their bounding box (diagonal D);
// x denotes an offset from P.  Source sub-tiles whose box lies within D/8 of
// the target box (the near field) are evaluated with double-float offsets,
// (hi_j - hi_i) + (lo_j - lo_i) where hi = (float)x and lo = (float)(x - hi),
// so close pairs keep full FP32 relative accuracy.  For all other sub-tiles
// (the far field) the squared separation is expanded as
// r^2 + eps^2 = (|x_i|^2 + eps^2) + |x_j|^2 - 2 x_i . x_j and the
// acceleration sum is split as sum_j s_ij m_j x_j - x_i sum_j s_ij m_j,
// s_ij = (r^2 + eps^2)^(-3/2): per far pair one add, seven FMAs, two
// multiplies and the rsqrt (eleven vector-ALU operations instead of
// thirteen).  Outside the near field |x_i|, |x_j| <= 5 r, which bounds the
// rounding error of both rewritings to a few units of 2^-24 per pair.  The
// two sums are kept apart (Kahan-compensated FP32 over tiles) and combined
// in FP64 at the end; near-field contributions are added to the first sum
// directly.  Each wavefront owns 64*IPL consecutive targets; the near/far
// choice of a sub-tile is uniform across the wavefront and tests the gap
// between the sub-tile's box and the box of the wavefront's own targets
// against D/8 of the workgroup box (the anchor's scale), so the bound above
// holds unchanged while fewer sub-tiles take the near-field path.
template <int TILE>
struct f32c_lds {
    float4 b[2][TILE];         // (-2 hi_x, -2 hi_y, -2 hi_z, |x|^2)
    float4 w[2][TILE];         // (m hi_x, m hi_y, m hi_z, m)
    float4 lo[2][TILE];        // (lo_x, lo_y, lo_z, 0)
    int near[2][kBlock / 64][TILE / kSub];   // per wavefront
};

// One workgroup task: targets ib .. ib + 256*IPL - 1 (sorted order) against
// sources [j0, j1).  Results go to particle order (order[]): final values
// (G applied, self potential removed) when final_out, else raw sums at
// ox[out_off + t] etc.
template <int IPL, int TILE, bool POT>
__device__ __attribute__((always_inline)) inline void f32c_task(
    f32c_lds<TILE>& L, const double* __restrict__ xs, const double* __restrict__ ys,
    const double* __restrict__ zs, const double* __restrict__ ms, const box6* __restrict__ sbox,
    const int32_t* __restrict__ order, int64_t n, int64_t ib, int64_t j0, int64_t j1, float eps2,
    double G, double inv_eps, int final_out, double* __restrict__ ox, double* __restrict__ oy,
    double* __restrict__ oz, double* __restrict__ op, int64_t out_off) {
    constexpr int kPer = (TILE + kBlock - 1) / kBlock;   // sources staged per lane
    const int tid = threadIdx.x;
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
    // this wavefront's targets: ib + wv*64*IPL .. + 64*IPL - 1, lane + 64 k;
    // their box from the IPL sub-tile boxes (the workgroup box if none is
    // in range)
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int64_t iw = ib + (int64_t)wv * 64 * IPL;
    box6 wb = bb;
    {
        const int64_t q0 = iw / kSub, nsub = (n + kSub - 1) / kSub;
        if (q0 < nsub) {
            wb = sbox[q0];
            for (int64_t q = q0 + 1; q < q0 + IPL && q < nsub; ++q) {
                const box6 o = sbox[q];
                for (int d = 0; d < 3; ++d) {
                    wb.lo[d] = o.lo[d] < wb.lo[d] ? o.lo[d] : wb.lo[d];
                    wb.hi[d] = o.hi[d] > wb.hi[d] ? o.hi[d] : wb.hi[d];
                }
            }
        }
    }

    float xh[IPL], yh[IPL], zh[IPL], xl[IPL], yl[IPL], zl[IPL], ck[IPL];
    float fx[IPL], fy[IPL], fz[IPL], f1[IPL], fp[IPL];
    kahan sx[IPL], sy[IPL], sz[IPL], s1[IPL], sp[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        int64_t i = iw + k * 64 + lane;
        if (i >= n) i = ib;
        const double dx = xs[i] - Px, dy = ys[i] - Py, dz = zs[i] - Pz;
        xh[k] = (float)dx;
        yh[k] = (float)dy;
        zh[k] = (float)dz;
        xl[k] = (float)(dx - (double)xh[k]);
        yl[k] = (float)(dy - (double)yh[k]);
        zl[k] = (float)(dz - (double)zh[k]);
        ck[k] = (float)(dx * dx + dy * dy + dz * dz + (double)eps2);
        sx[k] = sy[k] = sz[k] = s1[k] = sp[k] = kahan{0.0f, 0.0f};
    }

    // stage one tile of sources (and the near flags of its sub-tiles);
    // sources past j1 stage as massless points at the anchor
    auto stage = [&](int buf, int64_t jt) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int jl = u * kBlock + tid;
            if (jl >= TILE) break;
            const int64_t j = jt + jl;
            float4 b = make_float4(0.f, 0.f, 0.f, 0.f), w = b, l = b;
            if (j < j1) {
                const double dx = xs[j] - Px, dy = ys[j] - Py, dz = zs[j] - Pz;
                const float hx = (float)dx, hy = (float)dy, hz = (float)dz, m = (float)ms[j];
                b = make_float4(-2.0f * hx, -2.0f * hy, -2.0f * hz, (float)(dx * dx + dy * dy + dz * dz));
                w = make_float4(m * hx, m * hy, m * hz, m);
                l = make_float4((float)(dx - (double)hx), (float)(dy - (double)hy),
                                (float)(dz - (double)hz), 0.f);
            }
            L.b[buf][jl] = b;
            L.w[buf][jl] = w;
            L.lo[buf][jl] = l;
        }
        if (lane < TILE / kSub) {
            const int64_t q = jt / kSub + lane;
            int nr = 0;
            if (jt + (int64_t)lane * kSub < j1) nr = box_gap2(wb, sbox[q]) < near2;
            L.near[buf][wv][lane] = nr;
        }
    };

    stage(0, j0);
    __syncthreads();
    int cur = 0;
    for (int64_t jt = j0; jt < j1; jt += TILE) {
        const bool more = jt + TILE < j1;
#pragma unroll
        for (int k = 0; k < IPL; ++k) fx[k] = fy[k] = fz[k] = f1[k] = fp[k] = 0.0f;
        for (int sb = 0; sb < TILE / kSub; ++sb) {
            if (L.near[cur][wv][sb]) {
#pragma unroll 2
                for (int jj = sb * kSub; jj < (sb + 1) * kSub; ++jj) {
                    const float4 b = L.b[cur][jj];
                    const float4 ql = L.lo[cur][jj];
                    const float m = L.w[cur][jj].w;
                    // hi parts back from the B entries (scaling by -1/2 is exact)
                    const float qx = -0.5f * b.x, qy = -0.5f * b.y, qz = -0.5f * b.z;
#pragma unroll
                    for (int k = 0; k < IPL; ++k) {
                        const float dx = (qx - xh[k]) + (ql.x - xl[k]);
                        const float dy = (qy - yh[k]) + (ql.y - yl[k]);
                        const float dz = (qz - zh[k]) + (ql.z - zl[k]);
                        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2)));
                        const float rinv = __builtin_amdgcn_rsqf(r2);
                        const float mr = m * rinv;
                        const float s = mr * (rinv * rinv);
                        fx[k] = __builtin_fmaf(s, dx, fx[k]);
                        fy[k] = __builtin_fmaf(s, dy, fy[k]);
                        fz[k] = __builtin_fmaf(s, dz, fz[k]);
                        if (POT) fp[k] += mr;
                    }
                }
            } else {
#pragma unroll 4
                for (int jj = sb * kSub; jj < (sb + 1) * kSub; ++jj) {
                    const float4 b = L.b[cur][jj];
                    const float4 w = L.w[cur][jj];
#pragma unroll
                    for (int k = 0; k < IPL; ++k) {
                        const float r2 = __builtin_fmaf(xh[k], b.x, __builtin_fmaf(yh[k], b.y,
                                         __builtin_fmaf(zh[k], b.z, b.w + ck[k])));
                        const float rinv = __builtin_amdgcn_rsqf(r2);
                        const float s = (rinv * rinv) * rinv;
                        fx[k] = __builtin_fmaf(s, w.x, fx[k]);
                        fy[k] = __builtin_fmaf(s, w.y, fy[k]);
                        fz[k] = __builtin_fmaf(s, w.z, fz[k]);
                        f1[k] = __builtin_fmaf(s, w.w, f1[k]);
                        if (POT) fp[k] = __builtin_fmaf(rinv, w.w, fp[k]);
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
            sx[k].add(fx[k]);
            sy[k].add(fy[k]);
            sz[k].add(fz[k]);
            s1[k].add(f1[k]);
            if (POT) sp[k].add(fp[k]);
        }
        __syncthreads();                       // everyone is done with tile `cur`
        if (more) stage(cur ^ 1, jt + TILE);
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int64_t i = iw + k * 64 + lane;
        if (i >= n) continue;
        int32_t t = order[i];
        if ((uint64_t)t >= (uint64_t)n) continue;
        const double F1 = s1[k].value();
        const double gx = sx[k].value() - (double)xh[k] * F1;
        const double gy = sy[k].value() - (double)yh[k] * F1;
        const double gz = sz[k].value() - (double)zh[k] * F1;
        if (final_out) {
            ox[t] = G * gx;
            oy[t] = G * gy;
            oz[t] = G * gz;
            if (POT) op[t] = -G * (sp[k].value() - ms[i] * inv_eps);
        } else {
            const int64_t o = out_off + t;
            ox[o] = gx;
            oy[o] = gy;
            oz[o] = gz;
            if (POT) op[o] = sp[k].value();
        }
    }
    __syncthreads();                             // LDS free for the next task
}

template <int IPL, int TILE, bool POT>
__global__ __launch_bounds__(kBlock) void k_grav_f32c(
    const double* __restrict__ xs, const double* __restrict__ ys, const double* __restrict__ zs,
    const double* __restrict__ ms, const box6* __restrict__ sbox, const int32_t* __restrict__ order,
    int64_t n, int64_t jchunk, float eps2, double G, double inv_eps, int final_out,
    double* __restrict__ ox, double* __restrict__ oy, double* __restrict__ oz,
    double* __restrict__ op, int64_t ostride) {
    __shared__ f32c_lds<TILE> L;
    const int64_t j0 = (int64_t)blockIdx.y * jchunk;
    int64_t j1 = j0 + jchunk;
    if (j1 > n) j1 = n;
    f32c_task<IPL, TILE, POT>(L, xs, ys, zs, ms, sbox, order, n,
                              (int64_t)blockIdx.x * (kBlock * IPL), j0, j1, eps2, G, inv_eps,
                              final_out, ox, oy, oz, op, (int64_t)blockIdx.y * ostride);
}

// Persistent launch over the target blocks of several independent systems:
// each workgroup takes the next (system, block of 256*IPL targets) task from
// a counter until none is left; tasks are listed largest system first.
template <int IPL, int TILE, bool POT>
__global__ __launch_bounds__(kBlock) void k_grav_f32c_ens(const sg_ens_sys* __restrict__ sys,
                                                          const sg_ens_task* __restrict__ tasks,
                                                          int32_t ntasks, int32_t* counter,
                                                          float eps2, double G, double inv_eps) {
    __shared__ f32c_lds<TILE> L;
    __shared__ int32_t s_task;
    for (;;) {
        if (threadIdx.x == 0) s_task = atomicAdd(counter, 1);
        __syncthreads();
        // uniform: the task record and the system's pointers load into
        // scalar registers
        const int32_t t = __builtin_amdgcn_readfirstlane(s_task);
        __syncthreads();
        if (t >= ntasks) break;                  // every wavefront leaves here
        const sg_ens_task tk = tasks[t];
        const sg_ens_sys S = sys[tk.sys];
        f32c_task<IPL, TILE, POT>(L, S.xs, S.ys, S.zs, S.ms, (const box6*)S.sbox, S.order, S.n,
                                  (int64_t)tk.blk * (kBlock * IPL), 0, S.n, eps2, G, inv_eps, 1,
                                  S.gx, S.gy, S.gz, S.gp, 0);
    }
}

// FP64 form with the expanded far field (grav_variant 3, 4).  Same
// structure as the FP32C kernel: Morton-ordered targets and sources, an
// anchor P at the centre of the workgroup's target box, near-field source
// runs (box within D/8) in the difference form, far-field runs as
// r^2 + eps^2 = (|x_i|^2 + eps^2) + |x_j|^2 - 2 x_i . x_j and
// sum s m (x_j - x_i) = sum s (m x_j) - x_i sum s m, all in FP64 (no
// compensation needed).  Outside the near field |x| <= 5 r, so both
// rewritings cost a few units of 2^-53 per pair.  Per far pair: 1 add,
// 8 FMAs, 2 multiplies and the refined reciprocal square root, against
// 3 subtractions, 6 FMAs, 4 multiplies and 1 add in the difference form.
template <int TILE>
struct f64x_lds {
    d4 b[2][TILE];             // (-2 x, -2 y, -2 z, |x|^2), anchor-relative
    d4 w[2][TILE];             // (m x, m y, m z, m)
    int near[2][TILE / kSub];
};

template <int IPL, int TILE, bool POT, bool SEED32>
__global__ __launch_bounds__(kBlock) void k_grav_f64x(
    const double* __restrict__ xs, const double* __restrict__ ys, const double* __restrict__ zs,
    const double* __restrict__ ms, const box6* __restrict__ sbox, const int32_t* __restrict__ order,
    int64_t n, int64_t jchunk, double eps2, double G, double inv_eps, int final_out,
    double* __restrict__ ox, double* __restrict__ oy, double* __restrict__ oz,
    double* __restrict__ op, int64_t ostride) {
    constexpr int kPer = (TILE + kBlock - 1) / kBlock;   // sources staged per lane
    __shared__ f64x_lds<TILE> L;
    const int tid = threadIdx.x;
    const int64_t ib = (int64_t)blockIdx.x * (kBlock * IPL);
    const int64_t j0 = (int64_t)blockIdx.y * jchunk;
    int64_t j1 = j0 + jchunk;
    if (j1 > n) j1 = n;
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

    double xi[IPL], yi[IPL], zi[IPL], ck[IPL];
    double fx[IPL], fy[IPL], fz[IPL], f1[IPL], fp[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        int64_t i = ib + k * kBlock + tid;
        if (i >= n) i = ib;
        xi[k] = xs[i] - Px;
        yi[k] = ys[i] - Py;
        zi[k] = zs[i] - Pz;
        ck[k] = __builtin_fma(xi[k], xi[k], __builtin_fma(yi[k], yi[k], __builtin_fma(zi[k], zi[k], eps2)));
        fx[k] = fy[k] = fz[k] = f1[k] = fp[k] = 0.0;
    }
    // sources past j1 stage as massless points at the anchor
    auto stage = [&](int buf, int64_t jt) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int jl = u * kBlock + tid;
            if (jl >= TILE) break;
            const int64_t j = jt + jl;
            d4 b{0, 0, 0, 0}, w{0, 0, 0, 0};
            if (j < j1) {
                const double dx = xs[j] - Px, dy = ys[j] - Py, dz = zs[j] - Pz, m = ms[j];
                b = d4{-2.0 * dx, -2.0 * dy, -2.0 * dz,
                       __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz))};
                w = d4{m * dx, m * dy, m * dz, m};
            }
            L.b[buf][jl] = b;
            L.w[buf][jl] = w;
        }
        if (tid < TILE / kSub) {
            const int64_t q = jt / kSub + tid;
            int nr = 0;
            if (jt + (int64_t)tid * kSub < j1) nr = box_gap2(bb, sbox[q]) < near2;
            L.near[buf][tid] = nr;
        }
    };

    stage(0, j0);
    __syncthreads();
    int cur = 0;
    for (int64_t jt = j0; jt < j1; jt += TILE) {
        const bool more = jt + TILE < j1;
        for (int sb = 0; sb < TILE / kSub; ++sb) {
            if (L.near[cur][sb]) {
#pragma unroll 2
                for (int jj = sb * kSub; jj < (sb + 1) * kSub; ++jj) {
                    const d4 b = L.b[cur][jj];
                    const double m = L.w[cur][jj].w;
                    const double qx = -0.5 * b.x, qy = -0.5 * b.y, qz = -0.5 * b.z;   // exact
#pragma unroll
                    for (int k = 0; k < IPL; ++k) {
                        const double dx = qx - xi[k], dy = qy - yi[k], dz = qz - zi[k];
                        const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
                        const double rinv = rsqrt_f64<SEED32>(r2);
                        const double mr = m * rinv;
                        const double sv = mr * (rinv * rinv);
                        fx[k] = __builtin_fma(sv, dx, fx[k]);
                        fy[k] = __builtin_fma(sv, dy, fy[k]);
                        fz[k] = __builtin_fma(sv, dz, fz[k]);
                        if (POT) fp[k] += mr;
                    }
                }
            } else {
#pragma unroll 4
                for (int jj = sb * kSub; jj < (sb + 1) * kSub; ++jj) {
                    const d4 b = L.b[cur][jj];
                    const d4 w = L.w[cur][jj];
#pragma unroll
                    for (int k = 0; k < IPL; ++k) {
                        const double r2 = __builtin_fma(xi[k], b.x, __builtin_fma(yi[k], b.y,
                                          __builtin_fma(zi[k], b.z, b.w + ck[k])));
                        const double rinv = rsqrt_f64<SEED32>(r2);
                        const double sv = (rinv * rinv) * rinv;
                        fx[k] = __builtin_fma(sv, w.x, fx[k]);
                        fy[k] = __builtin_fma(sv, w.y, fy[k]);
                        fz[k] = __builtin_fma(sv, w.z, fz[k]);
                        f1[k] = __builtin_fma(sv, w.w, f1[k]);
                        if (POT) fp[k] = __builtin_fma(rinv, w.w, fp[k]);
                    }
                }
            }
        }
        __syncthreads();                       // everyone is done with tile `cur`
        if (more) stage(cur ^ 1, jt + TILE);
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int64_t i = ib + k * kBlock + tid;
        if (i >= n) continue;
        const int32_t t = order[i];
        if ((uint64_t)t >= (uint64_t)n) continue;
        const double gx = fx[k] - xi[k] * f1[k];
        const double gy = fy[k] - yi[k] * f1[k];
        const double gz = fz[k] - zi[k] * f1[k];
        if (final_out) {
            ox[t] = G * gx;
            oy[t] = G * gy;
            oz[t] = G * gz;
            if (POT) op[t] = -G * (fp[k] - ms[i] * inv_eps);
        } else {
            const int64_t o = (int64_t)blockIdx.y * ostride + t;
            ox[o] = gx;
            oy[o] = gy;
            oz[o] = gz;
            if (POT) op[o] = fp[k];
        }
    }
}

__global__ void k_counter_reset(int32_t* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

// Gather positions and masses into Morton order and build the bounding box
// of every run of kSub sorted particles (one wavefront per run): sorted
// index i of a launch whose blocks cover [0, n) in 256s.
__device__ inline void sorted_boxes_one(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ m, const int32_t* __restrict__ order, int64_t n, int64_t i,
    double* __restrict__ xs, double* __restrict__ ys, double* __restrict__ zs,
    double* __restrict__ ms, box6* __restrict__ sbox, uint32_t* __restrict__ err) {
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
        // every particle passes here once per preparation, also when the
        // Morton order (whose key pass checks positions too) is reused
        if (!(__builtin_isfinite(p[0]) && __builtin_isfinite(p[1]) && __builtin_isfinite(p[2])))
            atomicOr(err, SGE_GNONFINITE);
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

__global__ __launch_bounds__(kBlock) void k_sorted_boxes(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ m, const int32_t* __restrict__ order, int64_t n,
    double* __restrict__ xs, double* __restrict__ ys, double* __restrict__ zs,
    double* __restrict__ ms, box6* __restrict__ sbox, uint32_t* __restrict__ err) {
    sorted_boxes_one(x, y, z, m, order, n, (int64_t)blockIdx.x * kBlock + threadIdx.x, xs, ys, zs,
                     ms, sbox, err);
}

// The same for every system of an ensemble (blocks of 256 particles).
__global__ __launch_bounds__(kBlock) void k_seg_sorted_boxes(const sg_seg_sys* __restrict__ sys,
                                                             const int64_t* __restrict__ pfx,
                                                             int nsys) {
    int64_t lb;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &lb)];
    sorted_boxes_one(S.x, S.y, S.z, S.m, S.order, S.n, lb * kBlock + threadIdx.x, S.xs, S.ys,
                     S.zs, S.ms, (box6*)S.sbox, &S.g->err);
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

template <int IPL, int TILE, bool POT>
void launch_t(const sg_grav_args& a, dim3 grid, int64_t jchunk, int final_out, double* ox,
              double* oy, double* oz, double* op, int64_t ostride, hipStream_t st) {
    const double inv_eps = 1.0 / a.eps;
    if (a.precision == SG_FP32C)
        hipLaunchKernelGGL((k_grav_f32c<IPL, TILE, POT>), grid, dim3(kBlock), 0, st, a.xs, a.ys,
                           a.zs, a.ms, (const box6*)a.sbox, a.order, a.n, jchunk,
                           (float)(a.eps * a.eps), a.G, inv_eps, final_out, ox, oy, oz, op,
                           ostride);
    else if (a.variant == 3 || a.variant == 4) {
        if (a.variant == 3)
            hipLaunchKernelGGL((k_grav_f64x<IPL, TILE, POT, true>), grid, dim3(kBlock), 0, st,
                               a.xs, a.ys, a.zs, a.ms, (const box6*)a.sbox, a.order, a.n, jchunk,
                               a.eps * a.eps, a.G, inv_eps, final_out, ox, oy, oz, op, ostride);
        else
            hipLaunchKernelGGL((k_grav_f64x<IPL, TILE, POT, false>), grid, dim3(kBlock), 0, st,
                               a.xs, a.ys, a.zs, a.ms, (const box6*)a.sbox, a.order, a.n, jchunk,
                               a.eps * a.eps, a.G, inv_eps, final_out, ox, oy, oz, op, ostride);
    } else if (a.variant == 2)
        hipLaunchKernelGGL((k_grav_f64<IPL, TILE, POT, false>), grid, dim3(kBlock), 0, st, a.x,
                           a.y, a.z, a.m, a.n, jchunk, a.eps * a.eps, a.G, inv_eps, final_out, ox,
                           oy, oz, op, ostride);
    else
        hipLaunchKernelGGL((k_grav_f64<IPL, TILE, POT, true>), grid, dim3(kBlock), 0, st, a.x,
                           a.y, a.z, a.m, a.n, jchunk, a.eps * a.eps, a.G, inv_eps, final_out, ox,
                           oy, oz, op, ostride);
}

template <int IPL, int TILE>
void launch_pot(const sg_grav_args& a, dim3 grid, int64_t jchunk, int final_out, double* ox,
                double* oy, double* oz, double* op, int64_t ostride, hipStream_t st) {
    if (a.with_pot)
        launch_t<IPL, TILE, true>(a, grid, jchunk, final_out, ox, oy, oz, op, ostride, st);
    else
        launch_t<IPL, TILE, false>(a, grid, jchunk, final_out, ox, oy, oz, op, ostride, st);
}

template <int IPL>
void launch_tile(const sg_grav_args& a, dim3 grid, int64_t jchunk, int final_out, double* ox,
                 double* oy, double* oz, double* op, int64_t ostride, hipStream_t st) {
    switch (a.tile) {
        case 128: launch_pot<IPL, 128>(a, grid, jchunk, final_out, ox, oy, oz, op, ostride, st); break;
        case 512: launch_pot<IPL, 512>(a, grid, jchunk, final_out, ox, oy, oz, op, ostride, st); break;
        default: launch_pot<IPL, 256>(a, grid, jchunk, final_out, ox, oy, oz, op, ostride, st); break;
    }
}

template <int IPL, int TILE>
void launch_ens_pot(const sg_ens_sys* d_sys, const sg_ens_task* d_tasks, int32_t ntasks,
                    int32_t* d_counter, int with_pot, float eps2, double G, double inv_eps,
                    int nblocks, hipStream_t st) {
    if (with_pot)
        hipLaunchKernelGGL((k_grav_f32c_ens<IPL, TILE, true>), dim3(nblocks), dim3(kBlock), 0, st,
                           d_sys, d_tasks, ntasks, d_counter, eps2, G, inv_eps);
    else
        hipLaunchKernelGGL((k_grav_f32c_ens<IPL, TILE, false>), dim3(nblocks), dim3(kBlock), 0, st,
                           d_sys, d_tasks, ntasks, d_counter, eps2, G, inv_eps);
}

template <int IPL>
void launch_ens_tile(int tile, const sg_ens_sys* d_sys, const sg_ens_task* d_tasks, int32_t ntasks,
                     int32_t* d_counter, int with_pot, float eps2, double G, double inv_eps,
                     int nblocks, hipStream_t st) {
    switch (tile) {
        case 128: launch_ens_pot<IPL, 128>(d_sys, d_tasks, ntasks, d_counter, with_pot, eps2, G, inv_eps, nblocks, st); break;
        case 512: launch_ens_pot<IPL, 512>(d_sys, d_tasks, ntasks, d_counter, with_pot, eps2, G, inv_eps, nblocks, st); break;
        default: launch_ens_pot<IPL, 256>(d_sys, d_tasks, ntasks, d_counter, with_pot, eps2, G, inv_eps, nblocks, st); break;
    }
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
                             int32_t* d_counter, int with_pot, double eps, double G, int ipl,
                             int tile, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL(k_counter_reset, dim3(1), dim3(64), 0, st, d_counter);
    const float eps2 = (float)(eps * eps);
    const double inv_eps = 1.0 / eps;
    switch (ipl) {
        case 1: launch_ens_tile<1>(tile, d_sys, d_tasks, ntasks, d_counter, with_pot, eps2, G, inv_eps, nblocks, st); break;
        case 4: launch_ens_tile<4>(tile, d_sys, d_tasks, ntasks, d_counter, with_pot, eps2, G, inv_eps, nblocks, st); break;
        default: launch_ens_tile<2>(tile, d_sys, d_tasks, ntasks, d_counter, with_pot, eps2, G, inv_eps, nblocks, st); break;
    }
}

namespace {
template <int IPL, int TILE>
int occupancy_pot(int with_pot) {
    int nb = 0;
    const hipError_t e = with_pot
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_grav_f32c_ens<IPL, TILE, true>, kBlock, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_grav_f32c_ens<IPL, TILE, false>, kBlock, 0);
    return e == hipSuccess && nb > 0 ? nb : 1;
}
template <int IPL>
int occupancy_tile(int tile, int with_pot) {
    return tile == 128 ? occupancy_pot<IPL, 128>(with_pot)
                       : (tile == 512 ? occupancy_pot<IPL, 512>(with_pot) : occupancy_pot<IPL, 256>(with_pot));
}
}  // namespace

int sg_grav_ensemble_blocks_per_cu(int ipl, int tile, int with_pot) {
    return ipl == 1 ? occupancy_tile<1>(tile, with_pot)
                    : (ipl == 4 ? occupancy_tile<4>(tile, with_pot) : occupancy_tile<2>(tile, with_pot));
}

int sg_launch_grav_sorted(const sg_grav_args& a_in, hipStream_t st) {
    if (!a_in.order || !a_in.sorted || !a_in.x || !a_in.y || !a_in.z || !a_in.m || !a_in.err ||
        a_in.n < 1)
        return -1;
    sg_grav_args a = a_in;
    sorted_views(a);
    const unsigned nb = (unsigned)((a.n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_sorted_boxes, dim3(nb), dim3(kBlock), 0, st, a.x, a.y, a.z, a.m, a.order,
                       a.n, (double*)a.xs, (double*)a.ys, (double*)a.zs, (double*)a.ms,
                       (box6*)a.sbox, a.err);
    return 0;
}

void sg_seg_launch_grav_sorted(const sg_seg& s, hipStream_t st) {
    if (s.nblk[SG_SEG_N] > 0)
        hipLaunchKernelGGL(k_seg_sorted_boxes, dim3((unsigned)s.nblk[SG_SEG_N]), dim3(kBlock), 0,
                           st, s.sys, s.pfx + SG_SEG_N * (s.nsys + 1), s.nsys);
}

int sg_launch_gravity(const sg_grav_args& a_in, hipStream_t st) {
    if (!a_in.x || !a_in.y || !a_in.z || !a_in.m || !a_in.gx || !a_in.gy || !a_in.gz ||
        !a_in.gpot || !a_in.part || a_in.n < 1)
        return -1;
    const bool morton = a_in.precision == SG_FP32C || a_in.variant >= 3;
    if (morton && (!a_in.order || !a_in.sorted)) return -1;
    if (a_in.tile != 128 && a_in.tile != 256 && a_in.tile != 512) return -1;
    sg_grav_args a = a_in;
    if (morton) sorted_views(a);
    const int ipl = a.ipl == 1 || a.ipl == 2 ? a.ipl : 4;
    const int64_t per = (int64_t)kBlock * ipl;
    const int64_t iblocks = (a.n + per - 1) / per;
    int split = a.split < 1 ? 1 : a.split;
    // source chunk: a multiple of the tile, covering n in `split` pieces
    int64_t jchunk = (a.n + split - 1) / split;
    jchunk = (jchunk + a.tile - 1) / a.tile * a.tile;
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
    switch (ipl) {
        case 1: launch_tile<1>(a, grid, jchunk, final_out, ox, oy, oz, op, ostride, st); break;
        case 2: launch_tile<2>(a, grid, jchunk, final_out, ox, oy, oz, op, ostride, st); break;
        default: launch_tile<4>(a, grid, jchunk, final_out, ox, oy, oz, op, ostride, st); break;
    }
    if (!final_out) {
        const unsigned nb = (unsigned)((a.n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_grav_reduce, dim3(nb), dim3(kBlock), 0, st, a.part, a.m, a.n, split,
                           a.with_pot, a.G, 1.0 / a.eps, a.gx, a.gy, a.gz, a.gpot);
    }
    return 0;
}

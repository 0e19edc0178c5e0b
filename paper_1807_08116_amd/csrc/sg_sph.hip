// sg_sph.hip -- SPH sums over the neighbour lists (the paper's DC and HFC
// kernels, Sec. 3): density (Eq. SPH-mass-density with the cubic spline of
// Eq. SPH-Kernel), equation of state (Eq. e_p_rho), and the pressure +
// artificial-viscosity acceleration and energy rate (Eqs. dv_dt-SPH,
// de_dt-SPH, with the spiky kernel of Eq. SPH-Kernel-p for the gradient).
//
// Work is done on the gas gathered into sorted-slot order, so a target's
// neighbours are close in memory; results are scattered back to particle
// order.  The density and force passes walk a target's CSR row with a small
// group of lanes; the other passes take one thread per slot.
//
// FP64 form: every pair quantity in FP64.  FP32C form: the FP64 coordinate
// difference is rounded once to FP32 (cell-relative by construction: it is
// the difference itself), the rest of the pair arithmetic is FP32 and each
// sum is Kahan-compensated in FP32; results are returned in FP64.
#include "sg_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr double kPi = 3.14159265358979323846;

inline unsigned grid_for(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < 1 ? 1 : b);
}

// The density and force passes walk a target's neighbour row with
// kSphLanes lanes (every kSphLanes-th entry each) and combine the lanes'
// partial sums by an exchange over the group, in a fixed order, so each
// target's result is reproducible.  Eight lanes per target put eight
// independent record gathers in flight where one thread per target had
// one, and a wavefront's rows end within a few entries of each other.
// Measured at 2M particles (1M gas): density 0.51 -> 0.24 ms, the FP32C
// force pass (with its record build) 0.84 -> 0.56 ms, FP64 1.05 -> 0.66 ms
// (16 lanes: no faster; an LDS reservation that caps the workgroups per
// CU, which helped one thread per target, no longer does).  The XCDs take
// chunks of kSphChunk consecutive workgroups (2048 targets) in turn: as
// fast as plain launch order and 0.6x its fetched bytes, since a chunk's
// targets share neighbours in one L2 (one contiguous share of the slots
// per XCD measured slightly slower).
constexpr int kSphLanes = 8;
constexpr int64_t kSphChunk = 64;                  // workgroups per XCD chunk
constexpr int kSphTargets = kBlock / kSphLanes;     // targets per workgroup

inline unsigned grid_sph(int64_t ng) {
    int64_t b = (ng + kSphTargets - 1) / kSphTargets;
    return (unsigned)(b < 1 ? 1 : b);
}

// Sum of v over the kSphLanes lanes of this lane's group (butterfly; every
// lane of the group gets the same value).  All lanes of the wavefront call it.
__device__ inline double group_sum(double v) {
    for (int o = 1; o < kSphLanes; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct kahan {
    float s, c;
    __device__ inline void add(float v) {
        const float y = v - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ inline double value() const { return (double)s - (double)c; }
};

// Cubic spline shape (Eq. SPH-Kernel) without the 1/(pi h^3) factor.
template <typename T>
__device__ inline T spline_shape(T xi) {
    if (xi <= T(1)) return T(1) - T(1.5) * xi * xi + T(0.75) * xi * xi * xi;
    const T t = T(2) - xi;
    return t > T(0) ? T(0.25) * t * t * t : T(0);
}

// Density of target s from lane `sub` of its group; `valid` false for the
// groups past the end (they still take part in the group exchange).
__device__ inline void density_f64_lanes(const sg_sph_bufs& b, int64_t s, bool valid, int sub,
                                         double* __restrict__ rho_out) {
    double acc = 0.0;
    sg_prec pi{};
    if (valid) {
        pi = b.prec[s];
        if (sub == 0) acc = pi.m / (kPi * pi.h * pi.h * pi.h);   // self term m_i W(0, h_i)
        const int64_t e1 = b.nbr_off[s + 1];
        for (int64_t e = b.nbr_off[s] + sub; e < e1; e += kSphLanes) {
            const sg_prec pj = b.prec[b.nbr_idx[e]];
            const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double hij = 0.5 * (pi.h + pj.h);
            const double inv = 1.0 / hij;
            acc += pj.m * spline_shape(r * inv) * (inv * inv * inv) * (1.0 / kPi);
        }
    }
    acc = group_sum(acc);
    if (valid && sub == 0) {
        b.rho_s[s] = acc;
        rho_out[b.perm[s]] = acc;
    }
}

__global__ __launch_bounds__(kBlock) void k_density_f64(sg_sph_bufs b, const sg_grid_dev* g,
                                                        int64_t ng, double* __restrict__ rho_out) {
    if (g->err & (SGE_SORT_FATAL | SGE_NNZ)) return;
    const int64_t s = xcd_chunk_block(blockIdx.x, gridDim.x, kSphChunk) * kSphTargets + threadIdx.x / kSphLanes;
    density_f64_lanes(b, s, s < ng, threadIdx.x % kSphLanes, rho_out);
}

__device__ inline void density_f32_lanes(const sg_sph_bufs& b, int64_t s, bool valid, int sub,
                                         double* __restrict__ rho_out) {
    kahan acc{0.0f, 0.0f};
    if (valid) {
        const sg_prec pi = b.prec[s];
        const float hi = (float)pi.h;
        if (sub == 0) acc.s = (float)(pi.m / (kPi * pi.h * pi.h * pi.h));
        const int64_t e1 = b.nbr_off[s + 1];
        for (int64_t e = b.nbr_off[s] + sub; e < e1; e += kSphLanes) {
            const sg_prec pj = b.prec[b.nbr_idx[e]];
            const float dx = (float)(pi.x - pj.x), dy = (float)(pi.y - pj.y),
                        dz = (float)(pi.z - pj.z);
            const float r = sqrtf(dx * dx + dy * dy + dz * dz);
            const float hij = 0.5f * (hi + (float)pj.h);
            const float inv = 1.0f / hij;
            acc.add((float)pj.m * spline_shape(r * inv) * (inv * inv * inv) * (float)(1.0 / kPi));
        }
    }
    const double rho = group_sum(acc.value());
    if (valid && sub == 0) {
        b.rho_s[s] = rho;
        rho_out[b.perm[s]] = rho;
    }
}

__global__ __launch_bounds__(kBlock) void k_density_f32(sg_sph_bufs b, const sg_grid_dev* g,
                                                        int64_t ng, double* __restrict__ rho_out) {
    if (g->err & (SGE_SORT_FATAL | SGE_NNZ)) return;
    const int64_t s = xcd_chunk_block(blockIdx.x, gridDim.x, kSphChunk) * kSphTargets + threadIdx.x / kSphLanes;
    density_f32_lanes(b, s, s < ng, threadIdx.x % kSphLanes, rho_out);
}

// The velocities and energies the force pass should use (of the current or
// predicted state), packed in particle order: the record build then reads
// one 32-byte record per slot through the permutation instead of four
// scattered doubles (at 1M gas its fetched bytes fell from 573 MB to about
// 150 MB).
__device__ inline void pack_ve_one(int64_t i, const double* __restrict__ vx,
                                   const double* __restrict__ vy, const double* __restrict__ vz,
                                   const double* __restrict__ e, double* __restrict__ ve) {
    const double4 r = make_double4(vx[i], vy[i], vz[i], e[i]);
    reinterpret_cast<double4*>(ve)[i] = r;
}

__global__ __launch_bounds__(kBlock) void k_pack_ve(const sg_grid_dev* g, int64_t ng,
                                                    const double* __restrict__ vx,
                                                    const double* __restrict__ vy,
                                                    const double* __restrict__ vz,
                                                    const double* __restrict__ e,
                                                    double* __restrict__ ve) {
    if (g->err & (SGE_SORT_FATAL | SGE_NNZ)) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < ng) pack_ve_one(i, vx, vy, vz, e, ve);
}

// One record per slot of the packed state, with p / rho^2 and the sound
// speed sqrt(gamma p / rho) from the ideal-gas law.
__device__ inline void sph_prep_one(const sg_sph_bufs& b, int64_t s, int precision,
                                    double gamma) {
    const int32_t i = b.perm[s];
    const double4 v = reinterpret_cast<const double4*>(b.ve)[i];
    const sg_prec q = b.prec[s];
    const double rho = b.rho_s[s];
    const double p = (gamma - 1.0) * rho * v.w;
    const double P = p / (rho * rho);
    const double c = sqrt(gamma * p / rho);
    if (precision == SG_FP32C) {
        sg_frec32 r;
        r.x = q.x;
        r.y = q.y;
        r.z = q.z;
        r.h = (float)q.h;
        r.m = (float)q.m;
        r.vx = (float)v.x;
        r.vy = (float)v.y;
        r.vz = (float)v.z;
        r.rho = (float)rho;
        r.P = (float)P;
        r.c = (float)c;
        r.pad[0] = r.pad[1] = 0.0f;
        b.f32[s] = r;
    } else {
        b.f64[s] = sg_frec64{q.x, q.y, q.z, q.h, q.m, v.x, v.y, v.z, rho, P, c, 0.0};
    }
}

__global__ __launch_bounds__(kBlock) void k_sph_prep(sg_sph_bufs b, const sg_grid_dev* g,
                                                     int64_t ng, int precision, double gamma) {
    if (g->err & (SGE_SORT_FATAL | SGE_NNZ)) return;
    const int64_t s = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (s >= ng) return;
    sph_prep_one(b, s, precision, gamma);
}

__device__ inline void sph_force_f64_lanes(const sg_sph_bufs& b, int64_t s, bool valid, int sub,
                                           double alpha, double beta, double eta,
                                           double* __restrict__ asx, double* __restrict__ asy,
                                           double* __restrict__ asz, double* __restrict__ dedt) {
    const double kgrad = -45.0 / (64.0 * kPi);
    double sx = 0, sy = 0, sz = 0, se = 0;
    if (valid) {
        const sg_frec64 a = b.f64[s];
        const int64_t e1 = b.nbr_off[s + 1];
        for (int64_t e = b.nbr_off[s] + sub; e < e1; e += kSphLanes) {
            const sg_frec64 o = b.f64[b.nbr_idx[e]];
            const double dx = a.x - o.x, dy = a.y - o.y, dz = a.z - o.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;                       // coincident pair: no gradient
            const double r = sqrt(r2);
            const double hij = 0.5 * (a.h + o.h);
            const double inv = 1.0 / hij;
            const double q = 2.0 - r * inv;
            if (q <= 0.0) continue;
            const double dvx = a.vx - o.vx, dvy = a.vy - o.vy, dvz = a.vz - o.vz;
            const double rv = dx * dvx + dy * dvy + dz * dvz;
            double nu = 0.0;
            if (rv < 0.0) {
                const double mu = hij * rv / (r2 + eta * hij * hij);
                nu = mu * (beta * mu - alpha * 0.5 * (a.c + o.c)) / (0.5 * (a.rho + o.rho));
            }
            const double Pij = a.P + o.P + nu;
            // grad W_p = dW_p/dxi * r_ij / (|r_ij| h_ij) = gw * r_ij
            const double inv2 = inv * inv;
            const double gw = kgrad * q * q * (inv2 * inv2) / r;
            const double f = o.m * Pij * gw;
            sx -= f * dx;
            sy -= f * dy;
            sz -= f * dz;
            se += f * rv;
        }
    }
    sx = group_sum(sx);
    sy = group_sum(sy);
    sz = group_sum(sz);
    se = group_sum(se);
    if (valid && sub == 0) {
        const int32_t i = b.perm[s];
        asx[i] = sx;
        asy[i] = sy;
        asz[i] = sz;
        dedt[i] = 0.5 * se;
    }
}

__global__ __launch_bounds__(kBlock) void k_sph_force_f64(sg_sph_bufs b, const sg_grid_dev* g,
                                                          int64_t ng, double alpha, double beta,
                                                          double eta, double* __restrict__ asx,
                                                          double* __restrict__ asy,
                                                          double* __restrict__ asz,
                                                          double* __restrict__ dedt) {
    if (g->err & (SGE_SORT_FATAL | SGE_NNZ)) return;
    const int64_t s = xcd_chunk_block(blockIdx.x, gridDim.x, kSphChunk) * kSphTargets + threadIdx.x / kSphLanes;
    sph_force_f64_lanes(b, s, s < ng, threadIdx.x % kSphLanes, alpha, beta, eta, asx, asy, asz,
                        dedt);
}

__device__ inline void sph_force_f32_lanes(const sg_sph_bufs& b, int64_t s, bool valid, int sub,
                                           float alpha, float beta, float eta,
                                           double* __restrict__ asx, double* __restrict__ asy,
                                           double* __restrict__ asz, double* __restrict__ dedt) {
    const float kgrad = (float)(-45.0 / (64.0 * kPi));
    kahan sx{0, 0}, sy{0, 0}, sz{0, 0}, se{0, 0};
    if (valid) {
        const sg_frec32 a = b.f32[s];
        const int64_t e1 = b.nbr_off[s + 1];
        for (int64_t e = b.nbr_off[s] + sub; e < e1; e += kSphLanes) {
            const sg_frec32 o = b.f32[b.nbr_idx[e]];
            const float dx = (float)(a.x - o.x), dy = (float)(a.y - o.y),
                        dz = (float)(a.z - o.z);
            const float r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0f) continue;
            const float r = sqrtf(r2);
            const float hij = 0.5f * (a.h + o.h);
            const float inv = 1.0f / hij;
            const float q = 2.0f - r * inv;
            if (q <= 0.0f) continue;
            const float dvx = a.vx - o.vx, dvy = a.vy - o.vy, dvz = a.vz - o.vz;
            const float rv = dx * dvx + dy * dvy + dz * dvz;
            float nu = 0.0f;
            if (rv < 0.0f) {
                const float mu = hij * rv / (r2 + eta * hij * hij);
                nu = mu * (beta * mu - alpha * 0.5f * (a.c + o.c)) / (0.5f * (a.rho + o.rho));
            }
            const float Pij = a.P + o.P + nu;
            const float inv2 = inv * inv;
            const float gw = kgrad * q * q * (inv2 * inv2) / r;
            const float f = o.m * Pij * gw;
            sx.add(-f * dx);
            sy.add(-f * dy);
            sz.add(-f * dz);
            se.add(f * rv);
        }
    }
    // each lane's compensated sum is exact to FP32 rounding of its terms;
    // the group combines them in FP64
    const double vx = group_sum(sx.value()), vy = group_sum(sy.value());
    const double vz = group_sum(sz.value()), ve = group_sum(se.value());
    if (valid && sub == 0) {
        const int32_t i = b.perm[s];
        asx[i] = vx;
        asy[i] = vy;
        asz[i] = vz;
        dedt[i] = 0.5 * ve;
    }
}

__global__ __launch_bounds__(kBlock) void k_sph_force_f32(sg_sph_bufs b, const sg_grid_dev* g,
                                                          int64_t ng, float alpha, float beta,
                                                          float eta, double* __restrict__ asx,
                                                          double* __restrict__ asy,
                                                          double* __restrict__ asz,
                                                          double* __restrict__ dedt) {
    if (g->err & (SGE_SORT_FATAL | SGE_NNZ)) return;
    const int64_t s = xcd_chunk_block(blockIdx.x, gridDim.x, kSphChunk) * kSphTargets + threadIdx.x / kSphLanes;
    sph_force_f32_lanes(b, s, s < ng, threadIdx.x % kSphLanes, alpha, beta, eta, asx, asy, asz,
                        dedt);
}

// Density, EOS records and the FP32C force pass for every system of an
// ensemble (the density and force passes take blocks of kSphTargets gas
// slots per system, the records blocks of 256); the records take the
// current state, or the predicted one (predicted != 0).
__global__ __launch_bounds__(kBlock) void k_seg_density(const sg_seg_sys* __restrict__ sys,
                                                        const int64_t* __restrict__ pfx,
                                                        int nsys) {
    int64_t lb;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &lb)];
    if (S.g->err & (SGE_SORT_FATAL | SGE_NNZ)) return;
    const int64_t s = lb * kSphTargets + threadIdx.x / kSphLanes;
    density_f32_lanes(S.sph, s, s < S.ng, threadIdx.x % kSphLanes, S.rho);
}

__global__ __launch_bounds__(kBlock) void k_seg_pack_ve(const sg_seg_sys* __restrict__ sys,
                                                        const int64_t* __restrict__ pfx,
                                                        int nsys, int predicted) {
    int64_t lb;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &lb)];
    if (S.g->err & (SGE_SORT_FATAL | SGE_NNZ)) return;
    const int64_t i = lb * kBlock + threadIdx.x;
    if (i >= S.ng) return;
    if (predicted) pack_ve_one(i, S.vtx, S.vty, S.vtz, S.et, S.sph.ve);
    else pack_ve_one(i, S.vx, S.vy, S.vz, S.e, S.sph.ve);
}

__global__ __launch_bounds__(kBlock) void k_seg_sph_prep(const sg_seg_sys* __restrict__ sys,
                                                         const int64_t* __restrict__ pfx,
                                                         int nsys) {
    int64_t lb;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &lb)];
    if (S.g->err & (SGE_SORT_FATAL | SGE_NNZ)) return;
    const int64_t s = lb * kBlock + threadIdx.x;
    if (s >= S.ng) return;
    sph_prep_one(S.sph, s, SG_FP32C, S.gamma);
}

__global__ __launch_bounds__(kBlock) void k_seg_sph_force(const sg_seg_sys* __restrict__ sys,
                                                          const int64_t* __restrict__ pfx,
                                                          int nsys) {
    int64_t lb;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &lb)];
    if (S.g->err & (SGE_SORT_FATAL | SGE_NNZ)) return;
    const int64_t s = lb * kSphTargets + threadIdx.x / kSphLanes;
    sph_force_f32_lanes(S.sph, s, s < S.ng, threadIdx.x % kSphLanes, (float)S.alpha,
                        (float)S.beta, (float)S.eta, S.asx, S.asy, S.asz, S.dedt);
}

// Step control of Sec. 2.2.  CFL bound of Eq. (dt-stability) per gas slot,
// reduced to the minimum over slots with at least one neighbour: positive
// doubles order like their bit patterns, so an integer atomic min is exact
// and order-independent.
__global__ void k_cfl_init(unsigned long long* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = 0x7ff0000000000000ull;   // +inf
}

__global__ __launch_bounds__(kBlock) void k_cfl(sg_sph_bufs b, const sg_grid_dev* g, int64_t ng,
                                                double alpha, double beta, double eta,
                                                const double* __restrict__ qx,
                                                const double* __restrict__ qy,
                                                const double* __restrict__ qz,
                                                const double* __restrict__ dedt,
                                                unsigned long long* __restrict__ out) {
    if (g->err & (SGE_SORT_FATAL | SGE_NNZ)) return;
    const int64_t s = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    double dt = __builtin_inf();
    if (s < ng && b.nbr_off[s + 1] > b.nbr_off[s]) {
        const sg_frec64 a = b.f64[s];
        double smin = __builtin_inf(), cmax = 0.0, mumax = 0.0;
        for (int64_t e = b.nbr_off[s]; e < b.nbr_off[s + 1]; ++e) {
            const sg_frec64 o = b.f64[b.nbr_idx[e]];
            const double dx = a.x - o.x, dy = a.y - o.y, dz = a.z - o.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double r = sqrt(r2);
            smin = r < smin ? r : smin;
            const double cij = 0.5 * (a.c + o.c);
            cmax = cij > cmax ? cij : cmax;
            const double rv = dx * (a.vx - o.vx) + dy * (a.vy - o.vy) + dz * (a.vz - o.vz);
            if (rv < 0.0) {
                const double hij = 0.5 * (a.h + o.h);
                const double mu = fabs(hij * rv / (r2 + eta * hij * hij));
                mumax = mu > mumax ? mu : mumax;
            }
        }
        const int32_t i = b.perm[s];
        const double q = sqrt(qx[i] * qx[i] + qy[i] * qy[i] + qz[i] * qz[i]);
        const double den = cmax * (1.0 + 1.2 * alpha) + 1.2 * beta * mumax +
                           sqrt(smin * (q + fabs(dedt[i])));
        if (den > 0.0) dt = smin / den;
    }
    unsigned long long v = (unsigned long long)__builtin_bit_cast(long long, dt);
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    if ((threadIdx.x & 63) == 0) atomicMin(out, v);
}

__global__ void k_cfl_final(unsigned long long* out, double C) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double v = __builtin_bit_cast(double, (long long)*out);
        *(double*)out = C * v;
    }
}

// h_i = sigma (m_i / rho_i)^{1/3} (Sec. 2.2, after Eq. SPH-Kernel).
__global__ __launch_bounds__(kBlock) void k_update_h(sg_sph_bufs b, const sg_grid_dev* g,
                                                     int64_t ng, double sigma,
                                                     double* __restrict__ h) {
    if (g->err & (SGE_SORT_FATAL | SGE_NNZ)) return;
    const int64_t s = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (s >= ng) return;
    h[b.perm[s]] = sigma * cbrt(b.ms[s] / b.rho_s[s]);
}

}  // namespace

void sg_launch_density(const sg_sph_bufs& b, const sg_grid_dev* g, int64_t ng, int precision,
                       double* rho_out, hipStream_t st) {
    if (precision == SG_FP32C)
        hipLaunchKernelGGL(k_density_f32, dim3(grid_sph(ng)), dim3(kBlock), 0, st, b, g, ng, rho_out);
    else
        hipLaunchKernelGGL(k_density_f64, dim3(grid_sph(ng)), dim3(kBlock), 0, st, b, g, ng, rho_out);
}

void sg_launch_sph_prep(const sg_sph_bufs& b, const sg_grid_dev* g, int64_t ng, int precision,
                        double gamma, const double* vx, const double* vy, const double* vz,
                        const double* e, hipStream_t st) {
    hipLaunchKernelGGL(k_pack_ve, dim3(grid_for(ng)), dim3(kBlock), 0, st, g, ng, vx, vy, vz, e,
                       b.ve);
    hipLaunchKernelGGL(k_sph_prep, dim3(grid_for(ng)), dim3(kBlock), 0, st, b, g, ng, precision,
                       gamma);
}

void sg_launch_sph_force(const sg_sph_bufs& b, const sg_grid_dev* g, int64_t ng, int precision,
                         double alpha, double beta, double eta, double* asx, double* asy,
                         double* asz, double* dedt, hipStream_t st) {
    if (precision == SG_FP32C)
        hipLaunchKernelGGL(k_sph_force_f32, dim3(grid_sph(ng)), dim3(kBlock), 0, st, b, g, ng,
                           (float)alpha, (float)beta, (float)eta, asx, asy, asz, dedt);
    else
        hipLaunchKernelGGL(k_sph_force_f64, dim3(grid_sph(ng)), dim3(kBlock), 0, st, b, g, ng,
                           alpha, beta, eta, asx, asy, asz, dedt);
}

int64_t sg_sph_blocks(int64_t ng) { return (ng + kSphTargets - 1) / kSphTargets; }

void sg_seg_launch_density(const sg_seg& s, hipStream_t st) {
    if (s.nblk[SG_SEG_SPH] == 0) return;
    hipLaunchKernelGGL(k_seg_density, dim3((unsigned)s.nblk[SG_SEG_SPH]), dim3(kBlock), 0, st,
                       s.sys,
                       s.pfx + SG_SEG_SPH * (s.nsys + 1), s.nsys);
}

void sg_seg_launch_sph_state(const sg_seg& s, int predicted, hipStream_t st) {
    if (s.nblk[SG_SEG_NG] == 0) return;
    hipLaunchKernelGGL(k_seg_pack_ve, dim3((unsigned)s.nblk[SG_SEG_NG]), dim3(kBlock), 0, st,
                       s.sys, s.pfx + SG_SEG_NG * (s.nsys + 1), s.nsys, predicted);
    hipLaunchKernelGGL(k_seg_sph_prep, dim3((unsigned)s.nblk[SG_SEG_NG]), dim3(kBlock), 0, st,
                       s.sys, s.pfx + SG_SEG_NG * (s.nsys + 1), s.nsys);
    hipLaunchKernelGGL(k_seg_sph_force, dim3((unsigned)s.nblk[SG_SEG_SPH]), dim3(kBlock), 0, st,
                       s.sys,
                       s.pfx + SG_SEG_SPH * (s.nsys + 1), s.nsys);
}

void sg_launch_cfl(const sg_sph_bufs& b, const sg_grid_dev* g, int64_t ng, double alpha,
                   double beta, double eta, double C, const double* qx, const double* qy,
                   const double* qz, const double* dedt, double* out, hipStream_t st) {
    unsigned long long* o = (unsigned long long*)out;
    hipLaunchKernelGGL(k_cfl_init, dim3(1), dim3(64), 0, st, o);
    hipLaunchKernelGGL(k_cfl, dim3(grid_for(ng)), dim3(kBlock), 0, st, b, g, ng, alpha, beta, eta,
                       qx, qy, qz, dedt, o);
    hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(64), 0, st, o, C);
}

void sg_launch_update_h(const sg_sph_bufs& b, const sg_grid_dev* g, int64_t ng, double sigma,
                        double* h, hipStream_t st) {
    hipLaunchKernelGGL(k_update_h, dim3(grid_for(ng)), dim3(kBlock), 0, st, b, g, ng, sigma, h);
}

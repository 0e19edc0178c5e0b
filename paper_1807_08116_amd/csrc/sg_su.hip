// sg_su.hip -- the paper's SU kernel (Sec. 3) in its two states: the
// predictor of Eqs. (v-predictor), (e-predictor), (r-new) and the corrector
// of Eqs. (v-corrector), (e-corrector), always in FP64; the combination of
// the SPH and gravity parts into the total acceleration of Eq. (dv_dt-SPH);
// and FP64 conserved-quantity sums in a fixed reduction order.
#include "sg_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kDiagBlocks = 512;
constexpr int kDiag = 10;

inline unsigned grid_for(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < 1 ? 1 : b);
}

// Predictor of particle i (Eqs. v-predictor, e-predictor, r-new).
__device__ inline void predict_one(int64_t i, int64_t ng, double dt, double* __restrict__ x,
                                   double* __restrict__ y, double* __restrict__ z,
                                   const double* __restrict__ vx, const double* __restrict__ vy,
                                   const double* __restrict__ vz, const double* __restrict__ e,
                                   const double* __restrict__ ax, const double* __restrict__ ay,
                                   const double* __restrict__ az,
                                   const double* __restrict__ dedt, double* __restrict__ vtx,
                                   double* __restrict__ vty, double* __restrict__ vtz,
                                   double* __restrict__ et) {
    const double hdt = 0.5 * dt;
    const double ux = vx[i], uy = vy[i], uz = vz[i];
    const double wx = ux + dt * ax[i], wy = uy + dt * ay[i], wz = uz + dt * az[i];
    vtx[i] = wx;
    vty[i] = wy;
    vtz[i] = wz;
    x[i] += hdt * (wx + ux);
    y[i] += hdt * (wy + uy);
    z[i] += hdt * (wz + uz);
    if (i < ng) et[i] = e[i] + dt * dedt[i];
}

// Corrector of particle i (Eqs. v-corrector, e-corrector).
__device__ inline void correct_one(int64_t i, int64_t ng, double dt, double* __restrict__ vx,
                                   double* __restrict__ vy, double* __restrict__ vz,
                                   double* __restrict__ e, const double* __restrict__ vtx,
                                   const double* __restrict__ vty,
                                   const double* __restrict__ vtz,
                                   const double* __restrict__ et, const double* __restrict__ ax,
                                   const double* __restrict__ ay, const double* __restrict__ az,
                                   const double* __restrict__ dedt) {
    const double hdt = 0.5 * dt;
    vx[i] = 0.5 * (vx[i] + vtx[i]) + hdt * ax[i];
    vy[i] = 0.5 * (vy[i] + vty[i]) + hdt * ay[i];
    vz[i] = 0.5 * (vz[i] + vtz[i]) + hdt * az[i];
    if (i < ng) e[i] = 0.5 * (e[i] + et[i]) + hdt * dedt[i];
}

// a = a_SPH + g for gas (when an SPH part exists), a = g for halo.
__device__ inline void combine_one(int64_t i, int64_t ng, const double* __restrict__ asx,
                                   const double* __restrict__ asy,
                                   const double* __restrict__ asz,
                                   const double* __restrict__ gx, const double* __restrict__ gy,
                                   const double* __restrict__ gz, double* __restrict__ ax,
                                   double* __restrict__ ay, double* __restrict__ az) {
    double a0 = gx ? gx[i] : 0.0, a1 = gy ? gy[i] : 0.0, a2 = gz ? gz[i] : 0.0;
    if (asx && i < ng) {
        a0 += asx[i];
        a1 += asy[i];
        a2 += asz[i];
    }
    ax[i] = a0;
    ay[i] = a1;
    az[i] = a2;
}

__global__ __launch_bounds__(kBlock) void k_predict(
    int64_t n, int64_t ng, double dt, double* __restrict__ x, double* __restrict__ y,
    double* __restrict__ z, const double* __restrict__ vx, const double* __restrict__ vy,
    const double* __restrict__ vz, const double* __restrict__ e, const double* __restrict__ ax,
    const double* __restrict__ ay, const double* __restrict__ az, const double* __restrict__ dedt,
    double* __restrict__ vtx, double* __restrict__ vty, double* __restrict__ vtz,
    double* __restrict__ et) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    predict_one(i, ng, dt, x, y, z, vx, vy, vz, e, ax, ay, az, dedt, vtx, vty, vtz, et);
}

__global__ __launch_bounds__(kBlock) void k_correct(
    int64_t n, int64_t ng, double dt, double* __restrict__ vx, double* __restrict__ vy,
    double* __restrict__ vz, double* __restrict__ e, const double* __restrict__ vtx,
    const double* __restrict__ vty, const double* __restrict__ vtz,
    const double* __restrict__ et, const double* __restrict__ ax, const double* __restrict__ ay,
    const double* __restrict__ az, const double* __restrict__ dedt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    correct_one(i, ng, dt, vx, vy, vz, e, vtx, vty, vtz, et, ax, ay, az, dedt);
}

__global__ __launch_bounds__(kBlock) void k_combine(
    int64_t n, int64_t ng, const double* __restrict__ asx, const double* __restrict__ asy,
    const double* __restrict__ asz, const double* __restrict__ gx, const double* __restrict__ gy,
    const double* __restrict__ gz, double* __restrict__ ax, double* __restrict__ ay,
    double* __restrict__ az) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    combine_one(i, ng, asx, asy, asz, gx, gy, gz, ax, ay, az);
}

// The same three updates for every system of an ensemble in one launch
// (blocks of 256 particles per system).
__global__ __launch_bounds__(kBlock) void k_seg_predict(const sg_seg_sys* __restrict__ sys,
                                                        const int64_t* __restrict__ pfx,
                                                        int nsys, double dt) {
    int64_t lb;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &lb)];
    const int64_t i = lb * kBlock + threadIdx.x;
    if (i >= S.n) return;
    predict_one(i, S.ng, dt, S.x, S.y, S.z, S.vx, S.vy, S.vz, S.e, S.ax, S.ay, S.az, S.dedt,
                S.vtx, S.vty, S.vtz, S.et);
}

__global__ __launch_bounds__(kBlock) void k_seg_correct(const sg_seg_sys* __restrict__ sys,
                                                        const int64_t* __restrict__ pfx,
                                                        int nsys, double dt) {
    int64_t lb;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &lb)];
    const int64_t i = lb * kBlock + threadIdx.x;
    if (i >= S.n) return;
    correct_one(i, S.ng, dt, S.vx, S.vy, S.vz, S.e, S.vtx, S.vty, S.vtz, S.et, S.ax, S.ay, S.az,
                S.dedt);
}

// Both parts present (the ensemble's steady state): SPH for gas systems.
__global__ __launch_bounds__(kBlock) void k_seg_combine(const sg_seg_sys* __restrict__ sys,
                                                        const int64_t* __restrict__ pfx,
                                                        int nsys) {
    int64_t lb;
    const sg_seg_sys& S = sys[sg_seg_find(pfx, nsys, blockIdx.x, &lb)];
    const int64_t i = lb * kBlock + threadIdx.x;
    if (i >= S.n) return;
    const bool sph = S.ng > 0;
    combine_one(i, S.ng, sph ? S.asx : nullptr, sph ? S.asy : nullptr, sph ? S.asz : nullptr,
                S.gx, S.gy, S.gz, S.ax, S.ay, S.az);
}

__device__ inline void block_sum10(double (&v)[kDiag], double* sh) {
    // fixed-order tree over the block, one component at a time
    for (int c = 0; c < kDiag; ++c) {
        sh[threadIdx.x] = v[c];
        __syncthreads();
        for (int o = kBlock / 2; o > 0; o >>= 1) {
            if (threadIdx.x < (unsigned)o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        v[c] = sh[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_diag_partial(
    int64_t n, int64_t ng, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const double* __restrict__ vx, const double* __restrict__ vy,
    const double* __restrict__ vz, const double* __restrict__ m, const double* __restrict__ e,
    const double* __restrict__ pot, double* __restrict__ part) {
    __shared__ double sh[kBlock];
    double v[kDiag] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const double mi = m[i], ux = vx[i], uy = vy[i], uz = vz[i];
        const double px = x[i], py = y[i], pz = z[i];
        v[0] += 0.5 * mi * (ux * ux + uy * uy + uz * uz);
        if (i < ng) v[1] += mi * e[i];
        if (pot) v[2] += 0.5 * mi * pot[i];
        v[4] += mi * ux;
        v[5] += mi * uy;
        v[6] += mi * uz;
        v[7] += mi * (py * uz - pz * uy);
        v[8] += mi * (pz * ux - px * uz);
        v[9] += mi * (px * uy - py * ux);
    }
    block_sum10(v, sh);
    if (threadIdx.x == 0)
        for (int c = 0; c < kDiag; ++c) part[(int64_t)c * kDiagBlocks + blockIdx.x] = v[c];
}

__global__ __launch_bounds__(kBlock) void k_diag_final(const double* __restrict__ part,
                                                       double* __restrict__ out) {
    __shared__ double sh[kBlock];
    double v[kDiag];
    for (int c = 0; c < kDiag; ++c) {
        double s = 0;
        for (int b = threadIdx.x; b < kDiagBlocks; b += kBlock) s += part[c * kDiagBlocks + b];
        v[c] = s;
    }
    block_sum10(v, sh);
    if (threadIdx.x == 0) {
        for (int c = 0; c < kDiag; ++c) out[c] = v[c];
        out[3] = v[0] + v[1] + v[2];
    }
}

}  // namespace

void sg_launch_predict(int64_t n, int64_t ng, double dt, double* x, double* y, double* z,
                       const double* vx, const double* vy, const double* vz, const double* e,
                       const double* ax, const double* ay, const double* az, const double* dedt,
                       double* vtx, double* vty, double* vtz, double* et, hipStream_t st) {
    hipLaunchKernelGGL(k_predict, dim3(grid_for(n)), dim3(kBlock), 0, st, n, ng, dt, x, y, z, vx,
                       vy, vz, e, ax, ay, az, dedt, vtx, vty, vtz, et);
}

void sg_launch_correct(int64_t n, int64_t ng, double dt, double* vx, double* vy, double* vz,
                       double* e, const double* vtx, const double* vty, const double* vtz,
                       const double* et, const double* ax, const double* ay, const double* az,
                       const double* dedt, hipStream_t st) {
    hipLaunchKernelGGL(k_correct, dim3(grid_for(n)), dim3(kBlock), 0, st, n, ng, dt, vx, vy, vz,
                       e, vtx, vty, vtz, et, ax, ay, az, dedt);
}

void sg_launch_combine(int64_t n, int64_t ng, const double* asx, const double* asy,
                       const double* asz, const double* gx, const double* gy, const double* gz,
                       double* ax, double* ay, double* az, hipStream_t st) {
    hipLaunchKernelGGL(k_combine, dim3(grid_for(n)), dim3(kBlock), 0, st, n, ng, asx, asy, asz,
                       gx, gy, gz, ax, ay, az);
}

void sg_seg_launch_predict(const sg_seg& s, double dt, hipStream_t st) {
    if (s.nblk[SG_SEG_N] > 0)
        hipLaunchKernelGGL(k_seg_predict, dim3((unsigned)s.nblk[SG_SEG_N]), dim3(kBlock), 0, st,
                           s.sys, s.pfx + SG_SEG_N * (s.nsys + 1), s.nsys, dt);
}

void sg_seg_launch_correct(const sg_seg& s, double dt, hipStream_t st) {
    if (s.nblk[SG_SEG_N] > 0)
        hipLaunchKernelGGL(k_seg_correct, dim3((unsigned)s.nblk[SG_SEG_N]), dim3(kBlock), 0, st,
                           s.sys, s.pfx + SG_SEG_N * (s.nsys + 1), s.nsys, dt);
}

void sg_seg_launch_combine(const sg_seg& s, hipStream_t st) {
    if (s.nblk[SG_SEG_N] > 0)
        hipLaunchKernelGGL(k_seg_combine, dim3((unsigned)s.nblk[SG_SEG_N]), dim3(kBlock), 0, st,
                           s.sys, s.pfx + SG_SEG_N * (s.nsys + 1), s.nsys);
}

size_t sg_diag_tmp_bytes() { return sizeof(double) * kDiag * kDiagBlocks; }

void sg_launch_diagnostics(int64_t n, int64_t ng, const double* x, const double* y,
                           const double* z, const double* vx, const double* vy,
                           const double* vz, const double* m, const double* e,
                           const double* pot, double* tmp, double* out10, hipStream_t st) {
    hipLaunchKernelGGL(k_diag_partial, dim3(kDiagBlocks), dim3(kBlock), 0, st, n, ng, x, y, z,
                       vx, vy, vz, m, e, pot, tmp);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kBlock), 0, st, tmp, out10);
}

// Sparse-point kernels (gfx950): receiver interpolation (a gather, one thread
// per receiver), source injection (scatter with atomics, or a gather per
// target element), the standalone imaging kernels and the halo-zeroing kernel.  Paper: arXiv 1807.03032, Section 3.2 (eq. interp,
// Listing finject).
#include "fdw_device.h"

namespace fdw {

// ---------------------------------------------------------------------------
// Sparse kernels.  Interpolation: one thread per receiver (interp_receiver for
// linear weights).  Injection by scatter: one lane per support point of a
// source, atomics (sources may share points).
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) interp_kernel(SparseArgs a) {
    interp_receiver(a, blockIdx.x * blockDim.x + threadIdx.x);
}

// Receiver sampling for supports other than 4 or 8 points: one thread per
// receiver, corners summed in order.
__global__ void __launch_bounds__(256) interp_point_kernel(SparseArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.npoint) return;
    float v = 0.0f;
    for (int c = 0; c < a.ncorner; ++c) {
        float t = a.w[(int64_t)p * a.ncorner + c] * a.field[a.base[p] + corner_offset(a, c)];
        if (a.damp_mode == 2) t *= 1.0f + corner_damp(a, p, c);
        v += t;
    }
    a.rec_row[p] = v;
}

// Receiver rows of several shots in one launch: blockIdx.y selects the shot.
__global__ void __launch_bounds__(256) interp_multi_kernel(const SparseArgs *__restrict__ recs) {
    const SparseArgs &a = recs[blockIdx.y];
    interp_receiver(a, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void __launch_bounds__(256) inject_kernel(SparseArgs a) {
    const int lane = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = lane / a.ncorner;
    const int c = lane % a.ncorner;
    if (p >= a.npoint) return;
    const int64_t i = a.base[p] + corner_offset(a, c);
    float v = a.w[(int64_t)p * a.ncorner + c] * a.q_row[p] * fast_rcp(a.m[i]);
    if (a.damp_mode == 1) v /= 1.0f + corner_damp(a, p, c);
    atomicAdd(a.field + i, v);
}

// Injection as a gather, one thread per distinct target element: the same
// per-lane terms as inject_kernel (weights, point indices and the damping
// divisor gathered per target at operator creation, so that few loads depend
// on each other), summed in lane order and added once: no atomics, the same
// bits on every run.  Taken for many sparse points.
// A target's lanes are read four at a time (indices clamped to its last lane,
// so every load is in bounds and none waits on a branch), which keeps the
// loads of up to four lanes in flight together; the sum still runs in lane
// order.
__global__ void __launch_bounds__(256) inject_gather_kernel(SparseArgs a) {
#pragma clang fp contract(off)
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.ntarget) return;
    const int64_t i = a.tgt[j];
    const float f0 = a.field[i];  // this thread is the target's only writer
    const float rm = fast_rcp(a.m[i]);
    const float d = a.damp_mode == 1 ? a.gd[j] : 1.0f;
    const int k0 = a.goff[j], k1 = a.goff[j + 1];
    float acc = 0.0f;
    for (int k = k0; k < k1; k += 4) {
        float w[4], q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int kk = min(k + u, k1 - 1);
            w[u] = a.gw[kk];
            q[u] = a.q_row[a.gp[kk]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (k + u < k1) {
                float v = w[u] * q[u] * rm;
                if (a.damp_mode == 1) v /= d;
                acc += v;
            }
        }
    }
    a.field[i] = f0 + acc;
}

// Imaging condition of the adjoint-state gradient with respect to m, one
// thread per domain point:
//   grad += -nu [(u+ - 2u + u-)/dt^2 + eta (u+ - u-)/(2 dt)],  eta dt/2 = a.
template <int NDIM>
__global__ void __launch_bounds__(256) gradient_kernel(GradArgs a) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = NDIM == 3 ? (int)(blockIdx.y * blockDim.y + threadIdx.y) : 0;
    const int z = NDIM == 3 ? (int)blockIdx.z : (int)(blockIdx.y * blockDim.y + threadIdx.y);
    if (x >= a.g.nx || y >= a.g.ny || z >= a.g.nz) return;
    const int64_t i = a.g.off0 + (int64_t)z * a.g.sz + (int64_t)y * a.g.sy + x;
    const float damp = a.eta_x[x] + a.eta_z[z] + (NDIM == 3 ? a.eta_y[y] : 0.0f);
    const float un = a.u_next[i], uc = a.u_cur[i], up = a.u_prev[i];
    // (u+ - 2u + u-) + a (u+ - u-), divided by dt^2 (eta (u+ - u-)/(2 dt) = a (u+ - u-)/dt^2)
    const float s = ((un - uc) - (uc - up)) + damp * (un - up);
    a.grad[i] -= a.nu[i] * s * a.inv_dt2;
}

// Standalone imaging kernels, one thread per domain point, for the steps whose
// kernels do not fuse the imaging condition (2D grids, one-thread-per-point
// schedules, injections by the scatter kernel): the factor of a forward step
// from its three levels, and the update of the gradient from an adjoint level.
template <int NDIM>
__global__ void __launch_bounds__(256) imaging_factor_kernel(ImageArgs a) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = NDIM == 3 ? (int)(blockIdx.y * blockDim.y + threadIdx.y) : 0;
    const int z = NDIM == 3 ? (int)blockIdx.z : (int)(blockIdx.y * blockDim.y + threadIdx.y);
    if (x >= a.g.nx || y >= a.g.ny || z >= a.g.nz) return;
    const int64_t i = a.g.off0 + (int64_t)z * a.g.sz + (int64_t)y * a.g.sy + x;
    const float damp = damp_at(a.eta_x, a.eta_y, a.eta_z, NDIM, x, y, z);
    a.s_out[i] = imaging_factor(a.u_next[i], a.u_cur[i], a.u_prev[i], damp);
}

template <int NDIM>
__global__ void __launch_bounds__(256) image_update_kernel(ImageArgs a) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = NDIM == 3 ? (int)(blockIdx.y * blockDim.y + threadIdx.y) : 0;
    const int z = NDIM == 3 ? (int)blockIdx.z : (int)(blockIdx.y * blockDim.y + threadIdx.y);
    if (x >= a.g.nx || y >= a.g.ny || z >= a.g.nz) return;
    const int64_t i = a.g.off0 + (int64_t)z * a.g.sz + (int64_t)y * a.g.sy + x;
    a.grad[i] = image_update(a.grad[i], a.nu[i], a.s_in[i], a.inv_dt2);
}

// Writes zero to every element of one slot outside the domain.
__global__ void __launch_bounds__(256) zero_halo_kernel(int ndim, Geom g, int R, int64_t pitch_x,
                                                        int64_t pitch_y, int64_t planes, float *base) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = pitch_x * pitch_y * planes;
    if (e >= total) return;
    const int64_t xx = e % pitch_x;
    const int64_t row = e / pitch_x;
    const int64_t x = xx - (g.off0 % pitch_x);
    bool inside = x >= 0 && x < g.nx;
    if (ndim == 3) {
        const int64_t y = row % pitch_y - R;
        const int64_t z = row / pitch_y - R;
        inside = inside && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
    } else {
        const int64_t z = row - R;
        inside = inside && z >= 0 && z < g.nz;
    }
    if (!inside) base[e] = 0.0f;
}

// Logical array (x fastest, no halo) into the domain of a padded slot: one
// thread per logical element, x in a workgroup row.
__global__ void __launch_bounds__(256) pad_copy_kernel(Geom g, const float *__restrict__ src, float *dst) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int row = blockIdx.y * 4 + (threadIdx.x >> 6);  // y + ny * z
    if (x >= g.nx || row >= g.ny * g.nz) return;
    const int y = row % g.ny, z = row / g.ny;
    dst[g.off0 + (int64_t)z * g.sz + (int64_t)y * g.sy + x] = src[(int64_t)row * g.nx + x];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_inject(const SparseArgs &a, hipStream_t s) {
    if (a.npoint <= 0) return hipSuccess;
    if (a.ntarget > 0) {
        hipLaunchKernelGGL(inject_gather_kernel, dim3((unsigned)((a.ntarget + 255) / 256)), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    const int64_t lanes = (int64_t)a.npoint * a.ncorner;
    hipLaunchKernelGGL(inject_kernel, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_interp(const SparseArgs &a, hipStream_t s) {
    if (a.npoint <= 0) return hipSuccess;
    if (!interp_linear(a)) {
        hipLaunchKernelGGL(interp_point_kernel, dim3((unsigned)((a.npoint + 255) / 256)), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(interp_kernel, dim3((unsigned)((a.npoint + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_interp_multi(const SparseArgs *recs, int n, int64_t max_rec, hipStream_t s) {
    if (n <= 0 || max_rec <= 0) return hipSuccess;
    hipLaunchKernelGGL(interp_multi_kernel, dim3((unsigned)((max_rec + 255) / 256), (unsigned)n), dim3(256), 0, s,
                       recs);
    return hipGetLastError();
}

hipError_t launch_gradient(int ndim, const GradArgs &a, hipStream_t s) {
    dim3 blk(64, 4, 1);
    if (ndim == 3) {
        dim3 grd((a.g.nx + 63) / 64, (a.g.ny + 3) / 4, a.g.nz);
        hipLaunchKernelGGL(gradient_kernel<3>, grd, blk, 0, s, a);
    } else {
        dim3 grd((a.g.nx + 63) / 64, (a.g.nz + 3) / 4, 1);
        hipLaunchKernelGGL(gradient_kernel<2>, grd, blk, 0, s, a);
    }
    return hipGetLastError();
}

// one thread per domain point: 64 x 4 threads per workgroup
static void point_grid(int ndim, const Geom &g, dim3 &grd, dim3 &blk) {
    blk = dim3(64, 4, 1);
    grd = ndim == 3 ? dim3((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz) : dim3((g.nx + 63) / 64, (g.nz + 3) / 4, 1);
}

hipError_t launch_imaging_factor(int ndim, const ImageArgs &a, hipStream_t s) {
    dim3 grd, blk;
    point_grid(ndim, a.g, grd, blk);
    if (ndim == 3)
        hipLaunchKernelGGL(imaging_factor_kernel<3>, grd, blk, 0, s, a);
    else
        hipLaunchKernelGGL(imaging_factor_kernel<2>, grd, blk, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_image_update(int ndim, const ImageArgs &a, hipStream_t s) {
    dim3 grd, blk;
    point_grid(ndim, a.g, grd, blk);
    if (ndim == 3)
        hipLaunchKernelGGL(image_update_kernel<3>, grd, blk, 0, s, a);
    else
        hipLaunchKernelGGL(image_update_kernel<2>, grd, blk, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_zero_halo(int ndim, const Geom &g, int R, int64_t pitch_x, int64_t pitch_y, int64_t planes,
                            float *base, hipStream_t s) {
    const int64_t total = pitch_x * pitch_y * planes;
    hipLaunchKernelGGL(zero_halo_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, ndim, g, R,
                       pitch_x, pitch_y, planes, base);
    return hipGetLastError();
}

hipError_t launch_pad_copy(const Geom &g, const float *src, float *dst, hipStream_t s) {
    const int64_t rows = (int64_t)g.ny * g.nz;
    hipLaunchKernelGGL(pad_copy_kernel, dim3((unsigned)((g.nx + 63) / 64), (unsigned)((rows + 3) / 4)), dim3(256), 0,
                       s, g, src, dst);
    return hipGetLastError();
}

}  // namespace fdw

// Path tracker kernels (see track.hpp).  All arithmetic is complex FP64;
// the double-double endgame at t = 1 is the Newton corrector's.
#include <hip/hip_runtime.h>

#include <cmath>

#include "newton.hpp"
#include "track.hpp"

namespace pe {

namespace {

struct Cx {
    double re, im;
};

__device__ __forceinline__ Cx cmul(Cx a, Cx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ Cx cadd(Cx a, Cx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ Cx csub(Cx a, Cx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ Cx cscale(Cx a, double s) { return {a.re * s, a.im * s}; }

// z^e for an integer e >= 0 by repeated squaring
__device__ __forceinline__ Cx cpow(Cx z, int e)
{
    Cx r{1.0, 0.0};
    while (e > 0) {
        if (e & 1) r = cmul(r, z);
        z = cmul(z, z);
        e >>= 1;
    }
    return r;
}

__global__ void start_kernel(int64_t first, int64_t n_paths, int32_t n, const int32_t *deg,
                             double *xrh, double *xrl, double *xih, double *xil)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_paths) return;
    // mixed-radix digits of the path index, variable 0 fastest; the index
    // is taken modulo the product of the degrees as it goes
    uint64_t q = (uint64_t)(first + p);
    for (int i = 0; i < n; ++i) {
        const uint64_t d = (uint64_t)deg[i];
        const uint64_t k = q % d;
        q /= d;
        double s, c;
        sincospi(2.0 * (double)k / (double)d, &s, &c);
        xrh[p * n + i] = c;
        xrl[p * n + i] = 0.0;
        xih[p * n + i] = s;
        xil[p * n + i] = 0.0;
    }
}

__global__ void init_kernel(TrackArgs a, double h_init, double *xrl, double *xil)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = a.n_paths * a.n;
    if (e >= total) return;
    a.xs[0][e] = a.x[0][e];
    a.xs[1][e] = a.x[1][e];
    xrl[e] = 0.0;
    xil[e] = 0.0;
    if (e % a.n == 0) {
        const int64_t p = e / a.n;
        a.t[p] = 0.0;
        a.t1[p] = 0.0;
        a.h[p] = h_init;
        a.phase[p] = 0;
        a.succ[p] = 0;
        a.steps[p] = 0;
        a.status[p] = kRunning;
    }
}

// Entry e of the P x n x n Jacobians (column-major: column c, row i at
// c*n + i): H_x = tau * J_F + (1 - tau) * gamma * diag(d_i x_i^{d_i - 1});
// the threads of column 0 also write the right-hand side of row i.
__global__ void homotopy_kernel(TrackArgs a)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nn = (int64_t)a.n * a.n;
    if (e >= a.n_paths * nn) return;
    const int64_t p = e / nn;
    if (a.status[p] != kRunning) return;
    const int rem = (int)(e - p * nn);
    const int c = rem / a.n, i = rem - c * a.n;
    const bool predict = a.phase[p] == 0;
    const double tau = predict ? a.t[p] : a.t1[p];
    const Cx gamma{a.gamma_re, a.gamma_im};
    const Cx jf{a.J[0][e], a.J[1][e]};
    Cx hx = cscale(jf, tau);
    const bool diag = c == i, rhs = c == 0;
    if (diag || rhs) {
        const int64_t k = p * a.n + i;
        const Cx x{a.x[0][k], a.x[1][k]};
        const int d = a.deg[i];
        const Cx xd1 = cpow(x, d - 1);
        if (diag) hx = cadd(hx, cscale(cmul(gamma, cscale(xd1, (double)d)), 1.0 - tau));
        if (rhs) {
            const Cx g = csub(cmul(xd1, x), Cx{1.0, 0.0});
            const Cx f{a.f[0][k], a.f[1][k]};
            const Cx gg = cmul(gamma, g);
            // predictor: H_t = F - gamma G; corrector: H = tau F + (1 - tau) gamma G
            const Cx r = predict ? csub(f, gg) : cadd(cscale(f, tau), cscale(gg, 1.0 - tau));
            a.r[0][k] = r.re;
            a.r[1][k] = r.im;
        }
    }
    a.J[0][e] = hx.re;
    a.J[1][e] = hx.im;
}

// One wave per path.
__global__ __launch_bounds__(64) void step_kernel(TrackArgs a)
{
    const int64_t p = blockIdx.x;
    if (a.status[p] != kRunning) return;
    const int lane = threadIdx.x;
    const int n = a.n;
    const int64_t base = p * n;
    const int ph = a.phase[p];
    bool finite = true;
    int32_t status = kRunning;
    if (ph == 0) {
        // Euler predictor: dx/dt = -v with H_x v = H_t
        const double t = a.t[p];
        const double hh = fmin(a.h[p], 1.0 - t);
        for (int i = lane; i < n; i += 64) {
            const int64_t k = base + i;
            const double re = a.x[0][k] - hh * a.d[0][k];
            const double im = a.x[1][k] - hh * a.d[1][k];
            finite = finite && isfinite(re) && isfinite(im);
            a.x[0][k] = re;
            a.x[1][k] = im;
        }
        finite = __all(finite);
        if (lane == 0) {
            a.t1[p] = hh >= 1.0 - t ? 1.0 : t + hh;
            a.phase[p] = 1;
            a.steps[p] += 1;
            if (!finite) status = 3;
        }
    } else {
        // Newton corrector iteration ph at t1
        double nd = 0.0, nx = 0.0;
        for (int i = lane; i < n; i += 64) {
            const int64_t k = base + i;
            const double dre = a.d[0][k], dim = a.d[1][k];
            const double re = a.x[0][k] - dre, im = a.x[1][k] - dim;
            finite = finite && isfinite(re) && isfinite(im);
            a.x[0][k] = re;
            a.x[1][k] = im;
            nd = fmax(nd, hypot(dre, dim));
            nx = fmax(nx, hypot(re, im));
        }
        for (int off = 32; off >= 1; off >>= 1) {
            nd = fmax(nd, __shfl_xor(nd, off, 64));
            nx = fmax(nx, __shfl_xor(nx, off, 64));
        }
        finite = __all(finite);
        int decision;  // 0 continue, 1 accept, 2 reject
        if (!finite)
            decision = 3;
        else if (nd <= a.corr_tol * (1.0 + nx))
            decision = 1;
        else if (ph >= a.corr_iters)
            decision = 2;
        else
            decision = 0;
        if (decision == 1) {
            for (int i = lane; i < n; i += 64) {
                const int64_t k = base + i;
                a.xs[0][k] = a.x[0][k];
                a.xs[1][k] = a.x[1][k];
            }
        } else if (decision == 2) {
            for (int i = lane; i < n; i += 64) {
                const int64_t k = base + i;
                a.x[0][k] = a.xs[0][k];
                a.x[1][k] = a.xs[1][k];
            }
        }
        if (lane == 0) {
            if (decision == 3) {
                status = 3;
            } else if (decision == 1) {
                const double t = a.t1[p];
                a.t[p] = t;
                int s = a.succ[p] + 1;
                if (s >= 3) {
                    a.h[p] = fmin(2.0 * a.h[p], a.h_max);
                    s = 0;
                }
                a.succ[p] = s;
                a.phase[p] = 0;
                if (t >= 1.0) status = 0;
            } else if (decision == 2) {
                const double h = 0.5 * a.h[p];
                a.h[p] = h;
                a.succ[p] = 0;
                a.phase[p] = 0;
                if (h < a.h_min) status = kTrackStepUnderflow;
            } else {
                a.phase[p] = ph + 1;
            }
        }
    }
    if (lane == 0) {
        if (status == kRunning && a.phase[p] == 0 && a.steps[p] >= a.max_steps)
            status = kTrackStepLimit;
        if (status != kRunning)
            a.status[p] = status;
        else
            atomicAdd(a.running, 1);
    }
}

__global__ void endgame_kernel(int64_t n_paths, int32_t *tracked, int32_t *status)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_paths) return;
    const bool done = status[p] == 0;
    tracked[p] = done ? 1 : 0;
    if (done) status[p] = kRunning;
}

__global__ void end_kernel(int64_t n_paths, const int32_t *tracked, int32_t *status)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_paths) return;
    if (tracked[p] && status[p] != 0) status[p] = kTrackEndgameFailed;
}

unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_track_start(int64_t first, int64_t n_paths, int32_t n, const int32_t *deg,
                              double *const x[4], hipStream_t stream)
{
    if (n_paths <= 0) return hipSuccess;
    hipLaunchKernelGGL(start_kernel, dim3(blocks_for(n_paths, 256)), dim3(256), 0, stream, first,
                       n_paths, n, deg, x[0], x[1], x[2], x[3]);
    return hipGetLastError();
}

hipError_t launch_track_init(const TrackArgs &a, double h_init, double *const xlo[2],
                             hipStream_t stream)
{
    const int64_t total = a.n_paths * a.n;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(init_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, stream, a, h_init,
                       xlo[0], xlo[1]);
    return hipGetLastError();
}

hipError_t launch_track_homotopy(const TrackArgs &a, hipStream_t stream)
{
    const int64_t total = a.n_paths * (int64_t)a.n * a.n;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(homotopy_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_track_step(const TrackArgs &a, hipStream_t stream)
{
    if (a.n_paths <= 0) return hipSuccess;
    hipLaunchKernelGGL(step_kernel, dim3((unsigned)a.n_paths), dim3(64), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_track_endgame(int64_t n_paths, int32_t *tracked, int32_t *status,
                                hipStream_t stream)
{
    if (n_paths <= 0) return hipSuccess;
    hipLaunchKernelGGL(endgame_kernel, dim3(blocks_for(n_paths, 256)), dim3(256), 0, stream,
                       n_paths, tracked, status);
    return hipGetLastError();
}

hipError_t launch_track_end(int64_t n_paths, const int32_t *tracked, int32_t *status,
                            hipStream_t stream)
{
    if (n_paths <= 0) return hipSuccess;
    hipLaunchKernelGGL(end_kernel, dim3(blocks_for(n_paths, 256)), dim3(256), 0, stream, n_paths,
                       tracked, status);
    return hipGetLastError();
}

}  // namespace pe

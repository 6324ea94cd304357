// Convergence criterion of Sec. 5, Eq. (convergence_critertion): volume-weighted relative L2 change of
// rho, u (as a vector) and Tt between two states; uniform hex cells weigh 1
// (the weights cancel), cells of an unstructured mesh their volume.
// Two-stage fixed-order reduction (deterministic).
#include "gsis_common.h"
#include "gsis_launch.h"

#include <mutex>

namespace gsis {

__host__ __device__ inline int resid_blocks_of(const Geo &g) { return (g.ncell + 255) / 256; }
int resid_blocks(const Geo &g) { return resid_blocks_of(g); }

// red: the partial sums, [resid_blocks + 1][6] (the last row the total);
// nullptr means the case's own workspace buffer d.red.
__global__ __launch_bounds__(256) void k_resid_partial(GSIS_SPAN_ARGS, double *red)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    if (!red) red = d.red;
    int cell = blk * blockDim.x + threadIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};   // num rho, u, T; den rho, u, T
    if (cell < g.ncell && d.cflag[cell]) {
        const double *m = d.cm + (size_t)cell * NMOM;
        const double *p = d.snap + (size_t)cell * NSNAP;
        double dr = m[0] - p[0], dT = m[4] - p[4];
        v[0] = dr * dr;
        v[3] = p[0] * p[0];
        for (int a = 0; a < 3; ++a) {
            double du = m[1 + a] - p[1 + a];
            v[1] += du * du;
            v[4] += p[1 + a] * p[1 + a];
        }
        v[2] = dT * dT;
        v[5] = p[4] * p[4];
        if (d.uvol) {
            const double V = d.uvol[cell];
            for (int k = 0; k < 6; ++k) v[k] *= V;
        }
    }
    __shared__ double sh[6][256];
    for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 6; ++k) red[(size_t)blk * 6 + k] = sh[k][0];
}

// one block per case: the case's partial sums in block order
__global__ __launch_bounds__(256) void k_resid_final(GSIS_SPAN_ARGS, double *red)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Dev &d = C.d;
    if (!red) red = d.red;
    const int nblk = resid_blocks_of(C.g);
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
        for (int k = 0; k < 6; ++k) v[k] += red[(size_t)b * 6 + k];
    __shared__ double sh[6][256];
    for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int k = 0; k < 6; ++k) red[(size_t)nblk * 6 + k] = sh[k][0];
        if (d.hist) {
            const int it = *d.hist_ctr % d.hist_cap;
            double *h = d.hist + ((size_t)it * d.hist_ncase + d.hist_index) * 6;
            for (int k = 0; k < 6; ++k) h[k] = sh[k][0];
        }
    }
}

// advances the iteration counter of a batch's residual history
__global__ void k_hist_advance(int *ctr)
{
    if (threadIdx.x == 0) *ctr += 1;
}

hipError_t launch_hist_advance(int *ctr, hipStream_t s)
{
    hipLaunchKernelGGL(k_hist_advance, dim3(1), dim3(64), 0, s, ctr);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_snapshot(GSIS_SPAN_ARGS)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    int cell = blk * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    const double *m = d.cm + (size_t)cell * NMOM;
    double *p = d.snap + (size_t)cell * NSNAP;
    bool fl = d.cflag[cell] != 0;
    for (int k = 0; k < NSNAP; ++k) p[k] = fl ? m[k] : 0.0;
}

__global__ void k_zero_int(int *p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t launch_zero_int(int *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_int, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_residual(const Target &t, hipStream_t s, double *red)
{
    hipLaunchKernelGGL(k_resid_partial, dim3(t.nblk[K_CELL256]), dim3(256), 0, s, GSIS_SPAN(t.span(K_CELL256)), red);
    hipLaunchKernelGGL(k_resid_final, dim3(t.nblk[K_CASE]), dim3(256), 0, s, GSIS_SPAN(t.span(K_CASE)), red);
    return hipGetLastError();
}

// ------------------------------------------------ allocation-free residual
// The partial sums of gsis_residual_noalloc live in this file-scope array
// instead of the workspace: RESID_STATIC_BLOCKS blocks of 256 cells at most,
// plus the row of the total.  Each GPU holds its own copy until the process
// ends; every call on one GPU shares it, so calls that overlap on one GPU
// race.  Every slot a call reads was written by that call first (no
// clearing needed).
static __device__ __align__(256) double scratch[(RESID_STATIC_BLOCKS + 1) * 6];

// Device address of `scratch` on the current device, looked up once per
// device with that device current.  In host code the array's name is only a
// stand-in for the symbol: kernels and copies get this address.
hipError_t resid_static_scratch(double **out)
{
    constexpr int MAXDEV = 64;
    static std::mutex mu;
    static double *addr[MAXDEV] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAXDEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = (double *)p;
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_snapshot(const Target &t, hipStream_t s)
{
    hipLaunchKernelGGL(k_snapshot, dim3(t.nblk[K_CELL256]), dim3(256), 0, s, GSIS_SPAN(t.span(K_CELL256)));
    return hipGetLastError();
}

}  // namespace gsis

// VDF set-up kernels: boundary Maxwellian tables, initial Maxwellian,
// canonical <-> internal layout, and the pointwise GSIS update (Eq. updatef).
#include "gsis_common.h"
#include "gsis_launch.h"

#include <algorithm>

namespace gsis {

// M(1, u_b, T_b) at every node, per boundary slot, in the internal node order;
// mb1 = (dr/2) T_b M is the equilibrium of the rotational VDF.
__global__ void k_boundary_tables(Geo g, BcInfo bc, Dev d)
{
    int node = blockIdx.y * blockDim.x + threadIdx.x;
    int b = blockIdx.x;
    if (node >= g.nv) return;
    const double *t = d.nt64 + 4 * (size_t)node;
    double m = maxwell64(1.0, bc.u[b], bc.T[b], t[0], t[1], t[2]);
    double m1 = 0.5 * g.dr * bc.T[b] * m;
    size_t at = (size_t)b * g.nv + node;
    d.mb64[at] = m;
    d.mb32[at] = (float)m;
    d.mb1_64[at] = m1;
    d.mb1_32[at] = (float)m1;
}

// Incoming half-range moments of the boundary Maxwellian for slot b and
// face direction dir (outward normal n):  sum_{xi.n<0} w (xi.n) psi M(1,u_b,T_b),
// psi = (1, xi_x, xi_y, xi_z, |xi|^2 + (dr/2) T_b, (dr/2) T_b).
// One block per (b, dir); fixed-order tree reduction.
__global__ __launch_bounds__(256) void k_incoming_moments(Geo g, BcInfo bc, Dev d)
{
    int b = blockIdx.x / 6, dir = blockIdx.x % 6;
    int a = dir / 2;
    double sg = (dir & 1) ? 1.0 : -1.0;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    double h1 = 0.5 * g.dr * bc.T[b];
    for (int node = threadIdx.x; node < g.nv; node += blockDim.x) {
        const double *t = d.nt64 + 4 * (size_t)node;
        double x = t[0], y = t[1], z = t[2];
        double xn = sg * t[a];
        if (!(xn < 0.0)) continue;
        double w = t[3];
        double m = d.mb64[(size_t)b * g.nv + node];
        double ww = w * xn * m;
        acc[0] += ww;
        acc[1] += ww * x;
        acc[2] += ww * y;
        acc[3] += ww * z;
        acc[4] += ww * (x * x + y * y + z * z + h1);
        acc[5] += ww * h1;
    }
    __shared__ double sh[6][256];
    for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 6; ++k) d.inpsi[(b * 6 + dir) * 6 + k] = sh[k][0];
}

template <typename T>
__global__ void k_init_maxwellian(Geo g, Dev d, double rho, double ux, double uy, double uz, double Tt, double Tr)
{
    int node = blockIdx.y * blockDim.x + threadIdx.x;
    int cell = blockIdx.x;
    if (node >= g.nv) return;
    T *f0 = (T *)d.f0;
    T *f1 = (T *)d.f1;
    size_t at = (size_t)cell * g.nv + node;
    if (!d.cflag[cell]) {
        f0[at] = T(0);
        if (g.species == 1) f1[at] = T(0);
        return;
    }
    const double *t = d.nt64 + 4 * (size_t)node;
    double u[3] = {ux, uy, uz};
    double m = maxwell64(rho, u, Tt, t[0], t[1], t[2]);
    f0[at] = (T)m;
    if (g.species == 1) f1[at] = (T)(0.5 * g.dr * Tr * m);
}

template <typename T>
__global__ void k_to_canonical(Geo g, Dev d, const T *src, double *dst)
{
    int node = blockIdx.y * blockDim.x + threadIdx.x;
    int cell = blockIdx.x;
    if (node >= g.nv) return;
    size_t row = (size_t)cell * g.nv;
    dst[row + d.perm[node]] = (double)src[row + node];
}

template <typename T>
__global__ void k_from_canonical(Geo g, Dev d, const double *src, T *dst)
{
    int node = blockIdx.y * blockDim.x + threadIdx.x;
    int cell = blockIdx.x;
    if (node >= g.nv) return;
    size_t row = (size_t)cell * g.nv;
    dst[row + node] = d.cflag[cell] ? (T)src[row + d.perm[node]] : T(0);
}

// one internal node of every cell -> out[cell] (FP64)
template <typename T>
__global__ void k_vdf_node(Geo g, Dev d, int node, double *out)
{
    int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    out[cell] = (double)((const T *)d.f0)[(size_t)cell * g.nv + node];
}

// Eq. (updatef) pointwise (any node set): f0 += M(W') - M(W), f1 += (dr/2)[Tr' M(W') - Tr M(W)],
// both Maxwellians with the translational temperature.  The cell is uniform
// over the block: its prefactors rho (pi T)^{-3/2} and 1/T are computed once
// per wave, then one exponential per Maxwellian and point (the library's own
// FP64 exponential, clamped where it underflows).  A block covers a run of
// 256 nodes of one octant (blockIdx.y = octant * runs + run), so the octant's
// node counts are uniform over it.
template <typename T>
__global__ __launch_bounds__(256) void k_apply_correction(Geo g, Dev d, int nvb)
{
    const int cell = blockIdx.x;
    const int o = (int)blockIdx.y / nvb;
    const int l = ((int)blockIdx.y - o * nvb) * 256 + (int)threadIdx.x;
    if (l >= g.osize[o] || !d.cflag[cell]) return;
    const int node = g.obase[o] + l;
    const double *c = d.corr + (size_t)cell * NCORR;
    const double pn = PI * c[4], po = PI * c[10];
    const double an = c[0] / (pn * sqrt(pn)), ao = c[6] / (po * sqrt(po));
    const double itn = 1.0 / c[4], ito = 1.0 / c[10];
    const double *t = d.nt64 + 4 * (size_t)node;
    const double x = t[0], y = t[1], z = t[2];
    const double nx = x - c[1], ny = y - c[2], nz = z - c[3];
    const double ox = x - c[7], oy = y - c[8], oz = z - c[9];
    const double mn = an * exp_core(fmax(-(nx * nx + ny * ny + nz * nz) * itn, -745.0));
    const double mo = ao * exp_core(fmax(-(ox * ox + oy * oy + oz * oz) * ito, -745.0));
    size_t at = (size_t)cell * g.nv + node;
    T *f0 = (T *)d.f0;
    f0[at] = (T)((double)f0[at] + (mn - mo));
    if (g.species == 1) {
        T *f1 = (T *)d.f1;
        f1[at] = (T)((double)f1[at] + 0.5 * g.dr * (c[5] * mn - c[11] * mo));
    }
}

// The same update with the Maxwellians factored per axis: exp(-|xi - u|^2/T)
// = prod_a exp(-(xi_a - u_a)^2 / T), so one block per cell stages the 1-D
// factors of both Maxwellians in LDS (the prefactor folded into the x
// factor) and every point takes three products instead of two exponentials.
// Used on a tensor grid whose axes have at most CTAB nodes each.
constexpr int CTAB = 256;

template <typename T>
__global__ __launch_bounds__(256) void k_apply_correction_sep(Geo g, Dev d)
{
    __shared__ double ex[2][3][CTAB];
    const int cell = blockIdx.x;
    if (!d.cflag[cell]) return;   // uniform over the block
    const double *c = d.corr + (size_t)cell * NCORR;
    const double pn = PI * c[4], po = PI * c[10];
    const double an = c[0] / (pn * sqrt(pn)), ao = c[6] / (po * sqrt(po));
    const double itn = 1.0 / c[4], ito = 1.0 / c[10];
    const int n1x = g.n1[0], n1y = g.n1[1], span = g.n1[0] + g.n1[1] + g.n1[2];
    for (int e = threadIdx.x; e < 2 * span; e += blockDim.x) {
        const int m = e >= span, r = e - m * span;
        const int a = r < n1x ? 0 : (r < n1x + n1y ? 1 : 2);
        const int k = r - (a == 0 ? 0 : (a == 1 ? n1x : n1x + n1y));
        const double dx = d.xi64[a][k] - (m ? c[7 + a] : c[1 + a]);
        double v = exp_core(fmax(-dx * dx * (m ? ito : itn), -745.0));
        if (a == 0) v *= m ? ao : an;
        ex[m][a][k] = v;
    }
    __syncthreads();
    T *f0 = (T *)d.f0;
    T *f1 = (T *)d.f1;
    const bool dia = g.species == 1;
    const double h1 = 0.5 * g.dr;
    const size_t row = (size_t)cell * g.nv;
    for (int o = 0; o < 8; ++o) {
        const int nox = g.on[o][0], noy = g.on[o][1], n = g.osize[o];
        const int bx = (o & 1) ? 0 : g.k0[0], by = (o & 2) ? 0 : g.k0[1], bz = (o & 4) ? 0 : g.k0[2];
        for (int l = threadIdx.x; l < n; l += blockDim.x) {
            const int r = l / nox, lx = l - r * nox, lz = r / noy, ly = r - lz * noy;
            const int kx = bx + lx, ky = by + ly, kz = bz + lz;
            const double mn = ex[0][0][kx] * ex[0][1][ky] * ex[0][2][kz];
            const double mo = ex[1][0][kx] * ex[1][1][ky] * ex[1][2][kz];
            const size_t at = row + g.obase[o] + l;
            f0[at] = (T)((double)f0[at] + (mn - mo));
            if (dia) f1[at] = (T)((double)f1[at] + h1 * (c[5] * mn - c[11] * mo));
        }
    }
}

// ------------------------------------------------------------------ launches
// blockIdx.x = row (cell or boundary slot), blockIdx.y * 256 + tid = node
static dim3 node_grid(const Geo &g, int rows) { return dim3(rows, (g.nv + 255) / 256); }

hipError_t launch_setup_tables(const Geo &g, const BcInfo &bc, const Dev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_boundary_tables, node_grid(g, NBC), dim3(256), 0, s, g, bc, d);
    hipLaunchKernelGGL(k_incoming_moments, dim3(NBC * 6), dim3(256), 0, s, g, bc, d);
    return hipGetLastError();
}

hipError_t launch_init_maxwellian(const Geo &g, const Dev &d, bool fp32, double rho, const double *u, double Tt,
                                  double Tr, hipStream_t s)
{
    if (fp32)
        hipLaunchKernelGGL(k_init_maxwellian<float>, node_grid(g, g.ncell), dim3(256), 0, s, g, d, rho, u[0], u[1],
                           u[2], Tt, Tr);
    else
        hipLaunchKernelGGL(k_init_maxwellian<double>, node_grid(g, g.ncell), dim3(256), 0, s, g, d, rho, u[0], u[1],
                           u[2], Tt, Tr);
    return hipGetLastError();
}

hipError_t launch_to_canonical(const Geo &g, const Dev &d, bool fp32, const void *src, double *dst, hipStream_t s)
{
    if (fp32)
        hipLaunchKernelGGL(k_to_canonical<float>, node_grid(g, g.ncell), dim3(256), 0, s, g, d, (const float *)src, dst);
    else
        hipLaunchKernelGGL(k_to_canonical<double>, node_grid(g, g.ncell), dim3(256), 0, s, g, d, (const double *)src,
                           dst);
    return hipGetLastError();
}

hipError_t launch_from_canonical(const Geo &g, const Dev &d, bool fp32, const double *src, void *dst, hipStream_t s)
{
    if (fp32)
        hipLaunchKernelGGL(k_from_canonical<float>, node_grid(g, g.ncell), dim3(256), 0, s, g, d, src, (float *)dst);
    else
        hipLaunchKernelGGL(k_from_canonical<double>, node_grid(g, g.ncell), dim3(256), 0, s, g, d, src,
                           (double *)dst);
    return hipGetLastError();
}

hipError_t launch_vdf_node(const Geo &g, const Dev &d, bool fp32, int node, double *out, hipStream_t s)
{
    dim3 grd((g.ncell + 255) / 256);
    if (fp32) hipLaunchKernelGGL(k_vdf_node<float>, grd, dim3(256), 0, s, g, d, node, out);
    else hipLaunchKernelGGL(k_vdf_node<double>, grd, dim3(256), 0, s, g, d, node, out);
    return hipGetLastError();
}

hipError_t launch_apply_correction(const Geo &g, const Dev &d, bool fp32, hipStream_t s)
{
    if (!g.vlist && g.n1[0] <= CTAB && g.n1[1] <= CTAB && g.n1[2] <= CTAB) {
        if (fp32) hipLaunchKernelGGL(k_apply_correction_sep<float>, dim3(g.ncell), dim3(256), 0, s, g, d);
        else hipLaunchKernelGGL(k_apply_correction_sep<double>, dim3(g.ncell), dim3(256), 0, s, g, d);
        return hipGetLastError();
    }
    int omax = 0;
    for (int o = 0; o < 8; ++o) omax = std::max(omax, g.osize[o]);
    const int nvb = (omax + 255) / 256;
    if (8 * nvb > 65535) return hipErrorInvalidConfiguration;
    const dim3 grid(g.ncell, 8 * nvb);
    if (fp32)
        hipLaunchKernelGGL(k_apply_correction<float>, grid, dim3(256), 0, s, g, d, nvb);
    else
        hipLaunchKernelGGL(k_apply_correction<double>, grid, dim3(256), 0, s, g, d, nvb);
    return hipGetLastError();
}

}  // namespace gsis

// Second-order right-hand side of the kinetic update (Sec. 3.2).
//
// The interface values of the explicit flux divergence r^n of Eq.
// (delta_equations) are reconstructed from the upwind cell,
// f_up + phi_up grad f_up . (x_face - x_up), with a least-squares gradient
// over the fluid face neighbours and the Venkatakrishnan limiter phi; the
// increments on the left-hand side stay first-order upwind.  On the Cartesian
// grid the least-squares normal matrix is diagonal, so each gradient
// component is a central difference, one-sided next to a box face or a solid
// cell, and zero along an axis with no fluid neighbour.  Faces on the box or
// a solid surface keep first-order values (the cell's own value leaving, the
// boundary value entering), so the wall density balance is unchanged.
//
// The sweep keeps its first-order implicit operator in direct form; the
// difference of the two divergences, D2 - D1, moves to its right-hand side:
// it reads inv_dt f^n - (D2 - D1) per point from the buffer written here.
// Two passes over the VDF: the limiter of every point, then that term.
#include "gsis_common.h"
#include "gsis_launch.h"

#include <algorithm>

namespace gsis {

constexpr int RB = 256;      // nodes per block: one run of an octant
constexpr int RCELLS = 4;    // cells per block, consecutive in memory

// Block b of nblk: blocks are dealt to the 8 XCDs round robin, so logical
// block (b mod 8) (nblk / 8) + b / 8 gives every XCD one contiguous range of
// cells (x neighbours in the same L2).  Then: node run (octant o, run vb),
// and the first cell of the block.
struct ReconBlock { int o, l, cell0; };

__device__ __forceinline__ ReconBlock recon_block(const Geo &g, int nvb)
{
    const int nblk = (int)gridDim.x;
    int b = (int)blockIdx.x;
    if ((nblk & 7) == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
    const int ncr = (g.ncell + RCELLS - 1) / RCELLS;
    const int chunk = b / ncr, run = b - chunk * ncr;
    ReconBlock r;
    r.o = chunk / nvb;
    r.l = (chunk - r.o * nvb) * RB + (int)threadIdx.x;
    r.cell0 = run * RCELLS;
    return r;
}

// The face neighbours of a cell from its coordinates: index (the cell itself
// where there is none, so every load stays in range and none waits for a
// table) and whether it is a fluid cell; and, per axis, the second cell on
// the upwind side of octant o (the upwind neighbour's own upwind neighbour).
struct Around {
    int nb[6];
    bool has[6];
    int uu[3];
    bool huu[3];
};

__device__ __forceinline__ Around around(const Geo &g, const gptr<const int> &cflag, int cell, int o)
{
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int i = cell % nx, j = (cell / nx) % ny, k = cell / (nx * ny);
    const int co[3] = {i, j, k}, n[3] = {nx, ny, nz}, step[3] = {1, nx, nx * ny};
    Around a;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const bool lo = co[ax] > 0, hi = co[ax] < n[ax] - 1;
        a.nb[2 * ax] = lo ? cell - step[ax] : cell;
        a.nb[2 * ax + 1] = hi ? cell + step[ax] : cell;
        a.has[2 * ax] = lo && cflag[a.nb[2 * ax]];
        a.has[2 * ax + 1] = hi && cflag[a.nb[2 * ax + 1]];
        const int s = (o >> ax) & 1;   // 1: xi < 0, the upwind side is +
        const bool in2 = s ? co[ax] < n[ax] - 2 : co[ax] > 1;
        a.uu[ax] = in2 ? (s ? cell + 2 * step[ax] : cell - 2 * step[ax]) : cell;
        a.huu[ax] = in2 && (s ? a.has[2 * ax + 1] : a.has[2 * ax]) && cflag[a.uu[ax]];
    }
    return a;
}

// psi of Venkatakrishnan's limiter for a face: d2 = grad f . (x_face - x_c),
// D = (max or min of the neighbourhood) - f_c on the side of d2
template <typename T>
__device__ __forceinline__ T venkatakrishnan(T D, T d2, T e2)
{
    if (d2 == T(0)) return T(1);
    const T DD = D * D;
    return (DD + e2 + T(2) * D * d2) / (DD + T(2) * d2 * d2 + D * d2 + e2);
}

// least-squares gradient component from the cell value and its two neighbours
// along the axis (hm/hp: the neighbour is a fluid cell)
template <typename T>
__device__ __forceinline__ T lsq_component(T fm, T fc, T fp, bool hm, bool hp, T invh)
{
    if (hm && hp) return (fp - fm) * (T(0.5) * invh);
    if (hp) return (fp - fc) * invh;
    if (hm) return (fc - fm) * invh;
    return T(0);
}

template <typename T, bool DIA>
__global__ __launch_bounds__(RB) void k_recon_limiter(Geo g, Dev d, int nvb)
{
    const ReconBlock rb = recon_block(g, nvb);
    if (rb.o >= 8 || rb.l >= g.osize[rb.o]) return;
    const size_t nv = (size_t)g.nv, node = (size_t)g.obase[rb.o] + rb.l;
    const int ncell = g.ncell;
    const T e2 = (T)g.venk_e2;
    const gptr<const int> cflag = (gptr<const int>)d.cflag;
#pragma unroll
    for (int r = 0; r < RCELLS; ++r) {
        const int cell = min(rb.cell0 + r, ncell - 1);   // loads stay in range; the store is skipped
        const bool store = rb.cell0 + r < ncell && cflag[cell];
        const Around A = around(g, cflag, cell, rb.o);
#pragma unroll
        for (int q = 0; q < (DIA ? 2 : 1); ++q) {
            const gptr<const T> f = (gptr<const T>)(q ? d.f1 : d.f0);
            const T fc = f[(size_t)cell * nv + node];
            T fn[6];
#pragma unroll
            for (int dir = 0; dir < 6; ++dir) {
                const T v = f[(size_t)A.nb[dir] * nv + node];
                fn[dir] = A.has[dir] ? v : fc;
            }
            T phi = T(1);
            if (g.limited) {
                T mx = fc, mn = fc;
#pragma unroll
                for (int dir = 0; dir < 6; ++dir) { mx = fmax(mx, fn[dir]); mn = fmin(mn, fn[dir]); }
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const bool hm = A.has[2 * a], hp = A.has[2 * a + 1];
                    const T ga = lsq_component<T>(fn[2 * a], fc, fn[2 * a + 1], hm, hp, (T)g.invh[a]);
                    const T half = T(0.5) * (T)g.h[a];
                    if (hm) {
                        const T d2 = -ga * half;
                        phi = fmin(phi, venkatakrishnan<T>(d2 > T(0) ? mx - fc : mn - fc, d2, e2));
                    }
                    if (hp) {
                        const T d2 = ga * half;
                        phi = fmin(phi, venkatakrishnan<T>(d2 > T(0) ? mx - fc : mn - fc, d2, e2));
                    }
                }
            }
            if (store) {
                const gptr<T> lim = (gptr<T>)(q ? d.lim1 : d.lim0);
                lim[(size_t)cell * nv + node] = phi;
            }
        }
    }
}

// inv_dt f^n - (D2 - D1) per point.  Along axis a with upwind neighbour up
// (the octant fixes the direction for the whole block):
//   D2 - D1 = sum_a (xi_a / 2) (phi_c g_a,c [downwind face interior]
//                              - phi_up g_a,up [upwind face interior]),
// the reconstruction offsets of the leaving and the entering face values.
template <typename T, bool DIA>
__global__ __launch_bounds__(RB) void k_recon_source(Geo g, Dev d, int nvb)
{
    const ReconBlock rb = recon_block(g, nvb);
    if (rb.o >= 8 || rb.l >= g.osize[rb.o]) return;
    const size_t nv = (size_t)g.nv, node = (size_t)g.obase[rb.o] + rb.l;
    const int ncell = g.ncell;
    int kx, ky, kz;
    node_of(g, rb.o, rb.l, kx, ky, kz);
    constexpr bool F32 = sizeof(T) == 4;
    T xi[3];
    xi[0] = F32 ? (T)d.xi32[0][kx] : (T)d.xi64[0][kx];
    xi[1] = F32 ? (T)d.xi32[1][ky] : (T)d.xi64[1][ky];
    xi[2] = F32 ? (T)d.xi32[2][kz] : (T)d.xi64[2][kz];
    const T idt = (T)g.inv_dt;
    const gptr<const int> cflag = (gptr<const int>)d.cflag;
#pragma unroll
    for (int r = 0; r < RCELLS; ++r) {
        const int cell = min(rb.cell0 + r, ncell - 1);   // loads stay in range; the store is skipped
        const bool store = rb.cell0 + r < ncell && cflag[cell];
        const Around A = around(g, cflag, cell, rb.o);
#pragma unroll
        for (int q = 0; q < (DIA ? 2 : 1); ++q) {
            const gptr<const T> f = (gptr<const T>)(q ? d.f1 : d.f0);
            const gptr<const T> lim = (gptr<const T>)(q ? d.lim1 : d.lim0);
            const T fc = f[(size_t)cell * nv + node];
            const T phic = lim[(size_t)cell * nv + node];
            T corr = T(0);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int s = (rb.o >> a) & 1;            // 1: xi_a < 0, upwind is the + side
                const bool hm = A.has[2 * a], hp = A.has[2 * a + 1];
                const int up = s ? A.nb[2 * a + 1] : A.nb[2 * a];   // selects: no indexing by s
                const bool hup = s ? hp : hm, hdn = s ? hm : hp;
                const T invh = (T)g.invh[a];
                const T vm = f[(size_t)A.nb[2 * a] * nv + node];
                const T vp = f[(size_t)A.nb[2 * a + 1] * nv + node];
                const T vuu = f[(size_t)A.uu[a] * nv + node];
                const T phup = lim[(size_t)up * nv + node];
                const T fm = hm ? vm : fc, fp = hp ? vp : fc;
                const T gc = lsq_component<T>(fm, fc, fp, hm, hp, invh);
                T term = hdn ? phic * gc : T(0);
                if (hup) {
                    // the upwind cell's neighbours along a: this cell, and uu beyond it
                    const T fu = s ? fp : fm;
                    const T fuu = A.huu[a] ? vuu : fu;
                    const T gu = s ? lsq_component<T>(fc, fu, fuu, true, A.huu[a], invh)
                                   : lsq_component<T>(fuu, fu, fc, A.huu[a], true, invh);
                    term -= phup * gu;
                }
                corr += T(0.5) * xi[a] * term;
            }
            if (store) {
                const gptr<T> out = (gptr<T>)(q ? d.ho1 : d.ho0);
                out[(size_t)cell * nv + node] = idt * fc - corr;
            }
        }
    }
}

int recon_nvb(const Geo &g)
{
    int omax = 0;
    for (int o = 0; o < 8; ++o) omax = std::max(omax, g.osize[o]);
    return (omax + RB - 1) / RB;
}

hipError_t launch_recon(const Geo &g, const Dev &d, bool fp32, hipStream_t s)
{
    const int nvb = recon_nvb(g);
    const long long ncr = (g.ncell + RCELLS - 1) / RCELLS;
    const long long nblk = ncr * 8 * nvb;
    if (nblk <= 0 || nblk > 0x7fffffffll) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)nblk), block(RB);
    const bool dia = g.species == 1;
    if (fp32) {
        if (dia) {
            hipLaunchKernelGGL((k_recon_limiter<float, true>), grid, block, 0, s, g, d, nvb);
            hipLaunchKernelGGL((k_recon_source<float, true>), grid, block, 0, s, g, d, nvb);
        } else {
            hipLaunchKernelGGL((k_recon_limiter<float, false>), grid, block, 0, s, g, d, nvb);
            hipLaunchKernelGGL((k_recon_source<float, false>), grid, block, 0, s, g, d, nvb);
        }
    } else {
        if (dia) {
            hipLaunchKernelGGL((k_recon_limiter<double, true>), grid, block, 0, s, g, d, nvb);
            hipLaunchKernelGGL((k_recon_source<double, true>), grid, block, 0, s, g, d, nvb);
        } else {
            hipLaunchKernelGGL((k_recon_limiter<double, false>), grid, block, 0, s, g, d, nvb);
            hipLaunchKernelGGL((k_recon_source<double, false>), grid, block, 0, s, g, d, nvb);
        }
    }
    return hipGetLastError();
}

}  // namespace gsis

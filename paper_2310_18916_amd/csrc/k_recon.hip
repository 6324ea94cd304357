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
    const gptr<const int> nbr = (gptr<const int>)d.nbr;
    const gptr<const int> cflag = (gptr<const int>)d.cflag;
    for (int r = 0; r < RCELLS; ++r) {
        const int cell = rb.cell0 + r;
        if (cell >= ncell || !cflag[cell]) continue;   // uniform over the block
        int nb[6];
#pragma unroll
        for (int dir = 0; dir < 6; ++dir) nb[dir] = nbr[(size_t)dir * ncell + cell];
#pragma unroll
        for (int q = 0; q < (DIA ? 2 : 1); ++q) {
            const gptr<const T> f = (gptr<const T>)(q ? d.f1 : d.f0);
            const T fc = f[(size_t)cell * nv + node];
            T fn[6];
#pragma unroll
            for (int dir = 0; dir < 6; ++dir) fn[dir] = nb[dir] >= 0 ? f[(size_t)nb[dir] * nv + node] : fc;
            T phi = T(1);
            if (g.limited) {
                T mx = fc, mn = fc;
#pragma unroll
                for (int dir = 0; dir < 6; ++dir) { mx = fmax(mx, fn[dir]); mn = fmin(mn, fn[dir]); }
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const bool hm = nb[2 * a] >= 0, hp = nb[2 * a + 1] >= 0;
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
            const gptr<T> lim = (gptr<T>)(q ? d.lim1 : d.lim0);
            lim[(size_t)cell * nv + node] = phi;
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
    const gptr<const int> nbr = (gptr<const int>)d.nbr;
    const gptr<const int> cflag = (gptr<const int>)d.cflag;
    for (int r = 0; r < RCELLS; ++r) {
        const int cell = rb.cell0 + r;
        if (cell >= ncell || !cflag[cell]) continue;   // uniform over the block
        int nb[6], nn[3];
#pragma unroll
        for (int dir = 0; dir < 6; ++dir) nb[dir] = nbr[(size_t)dir * ncell + cell];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // second upwind neighbour: beyond the upwind one, same direction
            const int du = 2 * a + ((rb.o >> a) & 1);
            nn[a] = nb[du] >= 0 ? nbr[(size_t)du * ncell + nb[du]] : -1;
        }
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
                const int up = nb[2 * a + s], dn = nb[2 * a + 1 - s], uu = nn[a];
                const T invh = (T)g.invh[a];
                const T fm = nb[2 * a] >= 0 ? f[(size_t)nb[2 * a] * nv + node] : fc;
                const T fp = nb[2 * a + 1] >= 0 ? f[(size_t)nb[2 * a + 1] * nv + node] : fc;
                const T gc = lsq_component<T>(fm, fc, fp, nb[2 * a] >= 0, nb[2 * a + 1] >= 0, invh);
                T term = dn >= 0 ? phic * gc : T(0);
                if (up >= 0) {
                    // the upwind cell's neighbours along a: this cell, and uu beyond it
                    const T fu = s ? fp : fm;
                    const T fuu = uu >= 0 ? f[(size_t)uu * nv + node] : fu;
                    const T gu = s ? lsq_component<T>(fc, fu, fuu, true, uu >= 0, invh)
                                   : lsq_component<T>(fuu, fu, fc, uu >= 0, true, invh);
                    term -= lim[(size_t)up * nv + node] * gu;
                }
                corr += T(0.5) * xi[a] * term;
            }
            const gptr<T> out = (gptr<T>)(q ? d.ho1 : d.ho0);
            out[(size_t)cell * nv + node] = idt * fc - corr;
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

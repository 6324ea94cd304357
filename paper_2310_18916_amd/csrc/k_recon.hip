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

// A block walks one column of cells along z for one run of 256 nodes of one
// octant, keeping the z neighbours in registers (sliding windows), so the
// only neighbour loads are those of the four x and y neighbour columns,
// which the blocks of those columns read at about the same time.  Logical
// block = run * (nx ny) + column; blocks are dealt to the 8 XCDs round
// robin, so logical block (b mod 8) (nblk / 8) + b / 8 gives every XCD one
// contiguous range of columns.  Within a run the columns go in patches of
// RPX x RPY (where nx and ny divide), so that the y neighbours of a column
// are read by blocks RPX apart instead of nx apart and find their lines in
// the XCD's L2 (48^3 x 32^3 cavity, FP64: 65.0 -> 59.3 ms per pass).
constexpr int RPX = 8, RPY = 8;
struct ReconBlock { int o, l, col, i, j; };

__device__ __forceinline__ ReconBlock recon_block(const Geo &g, int nvb)
{
    const int nblk = (int)gridDim.x;
    int b = (int)blockIdx.x;
    if ((nblk & 7) == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
    const int ncol = g.nx * g.ny;
    const int chunk = b / ncol;
    ReconBlock r;
    const int rem = b - chunk * ncol;
    if (g.nx % RPX == 0 && g.ny % RPY == 0) {
        const int p = rem / (RPX * RPY), w = rem - p * (RPX * RPY);
        const int ppr = g.nx / RPX;
        r.i = (p % ppr) * RPX + w % RPX;
        r.j = (p / ppr) * RPY + w / RPX;
        r.col = r.i + g.nx * r.j;
    } else {
        r.col = rem;
        r.i = r.col % g.nx;
        r.j = r.col / g.nx;
    }
    r.o = chunk / nvb;
    r.l = (chunk - r.o * nvb) * RB + (int)threadIdx.x;
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

// Neighbours of a cell in the x and y directions from its coordinates: the
// index (the cell itself where there is none, so every load stays in range)
// and whether it is a fluid cell; per axis also the second cell on the
// upwind side of octant o.
struct AroundXY {
    int nb[4];
    bool has[4];
    int uu[2];
    bool huu[2];
};

__device__ __forceinline__ AroundXY around_xy(const Geo &g, const gptr<const int> &cflag, int cell, int i, int j, int o)
{
    const int co[2] = {i, j}, n[2] = {g.nx, g.ny}, step[2] = {1, g.nx};
    AroundXY a;
#pragma unroll
    for (int ax = 0; ax < 2; ++ax) {
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

// Venkatakrishnan phi of one point from the cell value and its six
// neighbours (value, and whether it is a fluid cell), x-, x+, y-, y+, z-, z+;
// e2 = (K h)^3, multiplied here by the square of the stencil's largest |f|.
template <typename T>
__device__ __forceinline__ T point_limiter(const Geo &g, T fc, const T *fv, const bool *has, T e2)
{
    T fn[6];
#pragma unroll
    for (int dir = 0; dir < 6; ++dir) fn[dir] = has[dir] ? fv[dir] : fc;
    T mx = fc, mn = fc;
#pragma unroll
    for (int dir = 0; dir < 6; ++dir) { mx = fmax(mx, fn[dir]); mn = fmin(mn, fn[dir]); }
    // the threshold relative to the local size of f: (K h)^3 S^2, S the largest |f| of the stencil
    const T S = fmax(fabs(mx), fabs(mn));
    e2 *= S * S;
    T phi = T(1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool hm = has[2 * a], hp = has[2 * a + 1];
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
    return phi;
}

// The reconstruction term of one axis:
//   (xi_a / 2) (phi_c g_a,c [downwind face interior] - phi_up g_a,up [upwind face interior])
// from the values along the axis: fm, fc, fp around the cell, fuu beyond the
// upwind neighbour, and the limiters of the cell and of the upwind neighbour.
template <typename T>
__device__ __forceinline__ T axis_term(int s, T xi, T invh, T fm, T fc, T fp, bool hm, bool hp, T fuu, bool huu,
                                       T phic, T phup)
{
    const bool hup = s ? hp : hm, hdn = s ? hm : hp;
    const T gc = lsq_component<T>(hm ? fm : fc, fc, hp ? fp : fc, hm, hp, invh);
    T term = hdn ? phic * gc : T(0);
    if (hup) {
        // the upwind cell's neighbours along the axis: this cell, and uu beyond it
        const T fu = s ? fp : fm;
        const T vuu = huu ? fuu : fu;
        const T gu = s ? lsq_component<T>(fc, fu, vuu, true, huu, invh)
                       : lsq_component<T>(vuu, fu, fc, huu, true, invh);
        term -= phup * gu;
    }
    return T(0.5) * xi * term;
}

template <typename T, bool DIA>
__global__ __launch_bounds__(RB) void k_recon_limiter(Geo g, Dev d, int nvb)
{
    constexpr int NQ = DIA ? 2 : 1;
    const ReconBlock rb = recon_block(g, nvb);
    if (rb.o >= 8 || rb.l >= g.osize[rb.o]) return;
    const size_t nv = (size_t)g.nv, node = (size_t)g.obase[rb.o] + rb.l;
    const int nz = g.nz, nxy = g.nx * g.ny;
    const T e2 = (T)g.venk_e2;
    const gptr<const int> cflag = (gptr<const int>)d.cflag;
    gptr<const T> f[NQ];
    gptr<T> lim[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        f[q] = (gptr<const T>)(q ? d.f1 : d.f0);
        lim[q] = (gptr<T>)(q ? d.lim1 : d.lim0);
    }
    // z window: the values at k - 1, k, k + 1 and their fluid flags
    T zm[NQ], zc[NQ], zp[NQ];
    bool fzm = false, fzc = cflag[rb.col] != 0, fzp = nz > 1 && cflag[rb.col + nxy] != 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        zc[q] = f[q][(size_t)rb.col * nv + node];
        zp[q] = f[q][(size_t)(nz > 1 ? rb.col + nxy : rb.col) * nv + node];
        zm[q] = zc[q];
    }
    for (int k = 0; k < nz; ++k) {
        const int cell = rb.col + k * nxy;
        const int ahead = k + 2 < nz ? cell + 2 * nxy : cell;   // the next window entry, issued first
        T nxt[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) nxt[q] = f[q][(size_t)ahead * nv + node];
        const bool fnx = k + 2 < nz && cflag[ahead] != 0;
        const AroundXY A = around_xy(g, cflag, cell, rb.i, rb.j, rb.o);
        if (fzc) {   // uniform over the block
            const bool has[6] = {A.has[0], A.has[1], A.has[2], A.has[3], k > 0 && fzm, k + 1 < nz && fzp};
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                T fv[6];
#pragma unroll
                for (int dir = 0; dir < 4; ++dir) fv[dir] = f[q][(size_t)A.nb[dir] * nv + node];
                fv[4] = zm[q];
                fv[5] = zp[q];
                const T phi = g.limited ? point_limiter<T>(g, zc[q], fv, has, e2) : T(1);
                lim[q][(size_t)cell * nv + node] = phi;
            }
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) { zm[q] = zc[q]; zc[q] = zp[q]; zp[q] = nxt[q]; }
        fzm = fzc; fzc = fzp; fzp = fnx;
    }
}

// inv_dt f^n - (D2 - D1) per point, the sum of axis_term over the three axes
// (the octant fixes the upwind side for the whole block).
template <typename T, bool DIA>
__global__ __launch_bounds__(RB) void k_recon_source(Geo g, Dev d, int nvb)
{
    constexpr int NQ = DIA ? 2 : 1;
    const ReconBlock rb = recon_block(g, nvb);
    if (rb.o >= 8 || rb.l >= g.osize[rb.o]) return;
    const size_t nv = (size_t)g.nv, node = (size_t)g.obase[rb.o] + rb.l;
    const int nz = g.nz, nxy = g.nx * g.ny;
    constexpr bool F32 = sizeof(T) == 4;
    const T xi0 = F32 ? (T)d.nt32[4 * node] : (T)d.nt64[4 * node];
    const T xi1 = F32 ? (T)d.nt32[4 * node + 1] : (T)d.nt64[4 * node + 1];
    const T xi2 = F32 ? (T)d.nt32[4 * node + 2] : (T)d.nt64[4 * node + 2];
    const T idt = (T)g.inv_dt;
    const int sz = (rb.o >> 2) & 1;   // 1: xi_z < 0, the z-upwind side is +
    const gptr<const int> cflag = (gptr<const int>)d.cflag;
    gptr<const T> f[NQ], lim[NQ];
    gptr<T> out[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        f[q] = (gptr<const T>)(q ? d.f1 : d.f0);
        lim[q] = (gptr<const T>)(q ? d.lim1 : d.lim0);
        out[q] = (gptr<T>)(q ? d.ho1 : d.ho0);
    }
    // z windows: f at k-2 .. k+2, the limiter at k-1 .. k+1, fluid flags at k-2 .. k+2
    auto row = [&](int k) -> size_t { return (size_t)(rb.col + min(max(k, 0), nz - 1) * nxy) * nv + node; };
    auto fl = [&](int k) -> bool { return k >= 0 && k < nz && cflag[rb.col + k * nxy] != 0; };
    T w[NQ][5], lw[NQ][3];
    unsigned wf = 0;   // bit m: the cell at k - 2 + m is a fluid cell
#pragma unroll
    for (int m = 0; m < 5; ++m) wf |= (unsigned)fl(m - 2) << m;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
#pragma unroll
        for (int m = 0; m < 5; ++m) w[q][m] = f[q][row(m - 2)];
#pragma unroll
        for (int m = 0; m < 3; ++m) lw[q][m] = lim[q][row(m - 1)];
    }
    for (int k = 0; k < nz; ++k) {
        const int cell = rb.col + k * nxy;
        // next window entries, issued first
        T nf[NQ], nl[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) { nf[q] = f[q][row(k + 3)]; nl[q] = lim[q][row(k + 2)]; }
        const bool nwf = fl(k + 3);
        const AroundXY A = around_xy(g, cflag, cell, rb.i, rb.j, rb.o);
        if (wf & 4u) {   // uniform over the block
            const bool hzm = (wf & 2u) != 0, hzp = (wf & 8u) != 0;
            const bool hzuu = sz ? (hzp && (wf & 16u)) : (hzm && (wf & 1u));
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const T fc = w[q][2];
                T vx[4], vuu[2], phup[2];
#pragma unroll
                for (int dir = 0; dir < 4; ++dir) vx[dir] = f[q][(size_t)A.nb[dir] * nv + node];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    vuu[a] = f[q][(size_t)A.uu[a] * nv + node];
                    const int s = (rb.o >> a) & 1;
                    phup[a] = lim[q][(size_t)(s ? A.nb[2 * a + 1] : A.nb[2 * a]) * nv + node];
                }
                const T phic = lw[q][1];
                T corr = axis_term<T>(rb.o & 1, xi0, (T)g.invh[0], vx[0], fc, vx[1], A.has[0], A.has[1], vuu[0],
                                      A.huu[0], phic, phup[0]);
                corr += axis_term<T>((rb.o >> 1) & 1, xi1, (T)g.invh[1], vx[2], fc, vx[3], A.has[2], A.has[3],
                                     vuu[1], A.huu[1], phic, phup[1]);
                corr += axis_term<T>(sz, xi2, (T)g.invh[2], w[q][1], fc, w[q][3], hzm, hzp,
                                     sz ? w[q][4] : w[q][0], hzuu, phic, sz ? lw[q][2] : lw[q][0]);
                out[q][(size_t)cell * nv + node] = idt * fc - corr;
            }
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
#pragma unroll
            for (int m = 0; m < 4; ++m) w[q][m] = w[q][m + 1];
            w[q][4] = nf[q];
            lw[q][0] = lw[q][1];
            lw[q][1] = lw[q][2];
            lw[q][2] = nl[q];
        }
        wf = (wf >> 1) | ((unsigned)nwf << 4);
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
    const long long nblk = (long long)g.nx * g.ny * 8 * nvb;
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

// Implicit first-order upwind kinetic update of Sec. 3.2, solved exactly.
//
// With first-order upwind fluxes on both sides of Eq. (delta_equations) the
// system for one velocity node is lower triangular in the node's upwind
// order, and for cell i
//   f_i^{n+1/2} = [f_i^n / dt + g_i / tau_i + sum_a a_a F_a] / (1/dt + 1/tau_i + sum_a a_a),
//   a_a = |xi_a| / h_a,
// where F_a is f^{n+1/2} of the upwind neighbour or the boundary value of the
// shared face.  Nodes of one octant share the upwind direction, so the
// domain is cut into TX x TY x TZ tiles in the octant's own frame and a launch
// processes one tile hyperplane tx + ty + tz = s for all 8 octants at once;
// a block owns one tile and a run of nodes of one octant (one node per
// thread, node-minor VDF layout, so every access is coalesced).  Inside the
// tile the thread walks cells in upwind order: the x-upwind value stays in a
// register, the y-upwind row in registers, the z-upwind plane in LDS (each
// thread touches only its own LDS column, so no barrier is needed).  Tile
// inflow faces are read from the VDF, which the upwind tile already holds
// in place.  The reference distribution is evaluated on the fly from FP64
// per-cell parameters (FP32 copies on the FP32 path), one exponential per
// Maxwellian shape.  Every cell's update has a fixed operand order, so the
// result is bitwise independent of the tile shape and of the schedule.
#include "gsis_common.h"
#include "gsis_launch.h"

namespace gsis {

template <typename T> struct Arith;
template <> struct Arith<float> {
    static __device__ __forceinline__ float ex(float x) { return __expf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return __fdividef(a, b); }
};
template <> struct Arith<double> {
    static __device__ __forceinline__ double ex(double x) { return exp(x); }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
};

struct SweepArgs {
    Geo g;
    void *f0, *f1;
    const void *par;
    const int *cflag, *nbr, *face_bc, *tiles;
    const void *fscale;
    const void *mb, *mb1;
    const void *xi[3];
};

// g / tau at node (cx, cy, cz) = xi - u of a monatomic cell
template <typename T>
__device__ __forceinline__ T ref_mono(const T *p, T cx, T cy, T cz)
{
    T c2 = cx * cx + cy * cy + cz * cz;
    T t = c2 * p[3];
    T E = p[4] * Arith<T>::ex(-t);
    T poly = p[5] + p[6] * cx + p[7] * cy + p[8] * cz + p[9] * c2 + (p[10] * cx + p[11] * cy + p[12] * cz) * (t - T(2.5));
    return E * poly;
}

// g0 / tau, g1 / tau of a diatomic cell (Rykov mixture of the four components)
template <typename T>
__device__ __forceinline__ void ref_dia(const T *p, T cx, T cy, T cz, T &g0, T &g1)
{
    T c2 = cx * cx + cy * cy + cz * cz;
    T tt = c2 * p[3], tr = c2 * p[4];
    T Et = p[5] * Arith<T>::ex(-tt);
    T Er = p[6] * Arith<T>::ex(-tr);
    T sht = (p[12] * cx + p[13] * cy + p[14] * cz) * (tt - T(2.5));
    T shr = (p[20] * cx + p[21] * cy + p[22] * cz) * (tr - T(2.5));
    T lt = p[7] + p[8] * cx + p[9] * cy + p[10] * cz + p[11] * c2;
    T lr = p[15] + p[16] * cx + p[17] * cy + p[18] * cz + p[19] * c2;
    T rt = p[23] * (T(1) + sht) + p[24] * cx + p[25] * cy + p[26] * cz + p[27];
    T rr = p[28] * (T(1) + shr) + p[29] * cx + p[30] * cy + p[31] * cz + p[32];
    g0 = Et * (lt + sht) + Er * (lr + shr);
    g1 = Et * rt + Er * rr;
}

template <typename T, int TX, int TY, bool DIA, bool RFN>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs A, int TZ, int plane_off, int nvb)
{
    extern __shared__ char smem_raw[];
    T *lds0 = (T *)smem_raw;
    T *lds1 = lds0 + TX * TY * blockDim.x;
    const Geo &g = A.g;
    const int b = blockIdx.x;
    const int vb = b % nvb;
    const int o = (b / nvb) & 7;
    const int t = b / (nvb * 8);
    const int l = vb * blockDim.x + threadIdx.x;
    if (l >= g.osize[o]) return;           // no barriers below: early exit is safe
    const int packed = A.tiles[plane_off + t];
    const int tx = packed & 0x3ff, ty = (packed >> 10) & 0x3ff, tz = (packed >> 20) & 0x3ff;
    const int sx = o & 1, sy = (o >> 1) & 1, sz = (o >> 2) & 1;
    int kxn, kyn, kzn;
    node_of(g, o, l, kxn, kyn, kzn);
    const T xix = ((const T *)A.xi[0])[kxn];
    const T xiy = ((const T *)A.xi[1])[kyn];
    const T xiz = ((const T *)A.xi[2])[kzn];
    const T ax = fabs(xix) * (T)g.invh[0];
    const T ay = fabs(xiy) * (T)g.invh[1];
    const T az = fabs(xiz) * (T)g.invh[2];
    const T idt = (T)g.inv_dt;
    const T den0 = idt + ax + ay + az;
    const int dxu = sx, dyu = 2 + sy, dzu = 4 + sz;   // upwind faces
    const size_t nv = (size_t)g.nv;
    const size_t node = (size_t)g.obase[o] + l;
    T *f0 = (T *)A.f0;
    T *f1 = (T *)A.f1;
    const T *par = (const T *)A.par;
    const T *fsc = (const T *)A.fscale;
    const T *mb = (const T *)A.mb;
    const T *mb1 = (const T *)A.mb1;
    const int ltid = threadIdx.x;
    const int bs = blockDim.x;

    auto bval0 = [&](int nb) -> T {
        int f = -nb - 1;
        return fsc[f] * mb[(size_t)A.face_bc[f] * nv + node];
    };
    auto bval1 = [&](int nb) -> T {
        int f = -nb - 1;
        return fsc[f] * mb1[(size_t)A.face_bc[f] * nv + node];
    };

    const int i0 = tx * TX, j0 = ty * TY, k0 = tz * TZ;
    for (int kz = 0; kz < TZ; ++kz) {
        const int kk = k0 + kz;
        if (kk >= g.nz) break;
        const int k = sz ? g.nz - 1 - kk : kk;
        T rowp0[TX], rowp1[TX];
        for (int ky = 0; ky < TY; ++ky) {
            const int jj = j0 + ky;
            if (jj >= g.ny) break;
            const int j = sy ? g.ny - 1 - jj : jj;
            T xp0 = T(0), xp1 = T(0);
#pragma unroll
            for (int kx = 0; kx < TX; ++kx) {
                const int ii = i0 + kx;
                if (ii >= g.nx) break;
                const int i = sx ? g.nx - 1 - ii : ii;
                const int cell = i + g.nx * (j + g.ny * k);
                if (!A.cflag[cell]) continue;
                const T *p = par + (size_t)cell * NPAR;
                const T cx = xix - p[0], cy = xiy - p[1], cz = xiz - p[2];
                T gt0, gt1 = T(0), invtau;
                if (DIA) {
                    ref_dia<T>(p, cx, cy, cz, gt0, gt1);
                    invtau = p[33];
                } else {
                    gt0 = ref_mono<T>(p, cx, cy, cz);
                    invtau = p[13];
                }
                const size_t at = (size_t)cell * nv + node;
                T num0 = gt0, num1 = gt1;
                if (RFN) {
                    num0 += idt * f0[at];
                    if (DIA) num1 += idt * f1[at];
                }
                const int *nbc = A.nbr + (size_t)cell * 6;
                const int lds_at = (ky * TX + kx) * bs + ltid;
                // x upwind
                T F0, F1 = T(0);
                int nb = nbc[dxu];
                if (nb >= 0) {
                    if (kx > 0) { F0 = xp0; if (DIA) F1 = xp1; }
                    else { F0 = f0[(size_t)nb * nv + node]; if (DIA) F1 = f1[(size_t)nb * nv + node]; }
                } else {
                    F0 = bval0(nb);
                    if (DIA) F1 = bval1(nb);
                }
                num0 += ax * F0;
                if (DIA) num1 += ax * F1;
                // y upwind
                nb = nbc[dyu];
                if (nb >= 0) {
                    if (ky > 0) { F0 = rowp0[kx]; if (DIA) F1 = rowp1[kx]; }
                    else { F0 = f0[(size_t)nb * nv + node]; if (DIA) F1 = f1[(size_t)nb * nv + node]; }
                } else {
                    F0 = bval0(nb);
                    if (DIA) F1 = bval1(nb);
                }
                num0 += ay * F0;
                if (DIA) num1 += ay * F1;
                // z upwind
                nb = nbc[dzu];
                if (nb >= 0) {
                    if (kz > 0) { F0 = lds0[lds_at]; if (DIA) F1 = lds1[lds_at]; }
                    else { F0 = f0[(size_t)nb * nv + node]; if (DIA) F1 = f1[(size_t)nb * nv + node]; }
                } else {
                    F0 = bval0(nb);
                    if (DIA) F1 = bval1(nb);
                }
                num0 += az * F0;
                if (DIA) num1 += az * F1;
                const T den = den0 + invtau;
                const T v0 = Arith<T>::div(num0, den);
                f0[at] = v0;
                xp0 = v0;
                rowp0[kx] = v0;
                lds0[lds_at] = v0;
                if (DIA) {
                    const T v1 = Arith<T>::div(num1, den);
                    f1[at] = v1;
                    xp1 = v1;
                    rowp1[kx] = v1;
                    lds1[lds_at] = v1;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ launches
struct Shape { int tx, ty; };
// compiled (tx, ty) per precision; tz is a run-time loop length
static const Shape kShapes32[] = {{4, 4}, {8, 8}, {16, 8}};
static const Shape kShapes64[] = {{4, 4}, {8, 4}, {8, 8}};

template <typename T, int TX, int TY>
static void sweep_plane(const SweepArgs &a, bool dia, bool rfn, int tz, int off, int ntile, int nvb, int bs,
                        hipStream_t s)
{
    size_t shm = (size_t)TX * TY * bs * sizeof(T) * (dia ? 2 : 1);
    dim3 grid((unsigned)(ntile * 8 * nvb));
    if (dia) {
        if (rfn) hipLaunchKernelGGL((k_sweep<T, TX, TY, true, true>), grid, dim3(bs), shm, s, a, tz, off, nvb);
        else hipLaunchKernelGGL((k_sweep<T, TX, TY, true, false>), grid, dim3(bs), shm, s, a, tz, off, nvb);
    } else {
        if (rfn) hipLaunchKernelGGL((k_sweep<T, TX, TY, false, true>), grid, dim3(bs), shm, s, a, tz, off, nvb);
        else hipLaunchKernelGGL((k_sweep<T, TX, TY, false, false>), grid, dim3(bs), shm, s, a, tz, off, nvb);
    }
}

bool sweep_shape_supported(bool fp32, int tx, int ty)
{
    if (fp32) {
        for (const Shape &s : kShapes32) if (s.tx == tx && s.ty == ty) return true;
    } else {
        for (const Shape &s : kShapes64) if (s.tx == tx && s.ty == ty) return true;
    }
    return false;
}

int sweep_shapes(bool fp32, int *out, int max)
{
    int n = 0;
    const Shape *sh = fp32 ? kShapes32 : kShapes64;
    int cnt = fp32 ? (int)(sizeof(kShapes32) / sizeof(Shape)) : (int)(sizeof(kShapes64) / sizeof(Shape));
    for (int k = 0; k < cnt && n < max; ++k) {
        out[2 * n] = sh[k].tx;
        out[2 * n + 1] = sh[k].ty;
        ++n;
    }
    return n;
}

hipError_t launch_sweep(const Geo &g, const Dev &d, bool fp32, int tx, int ty, int tz, int bs,
                        const int *plane_off, const int *plane_cnt, int nplane, hipStream_t s)
{
    SweepArgs a;
    a.g = g;
    a.f0 = d.f0;
    a.f1 = d.f1;
    a.par = fp32 ? (const void *)d.parf : (const void *)d.par;
    a.cflag = d.cflag;
    a.nbr = d.nbr;
    a.face_bc = d.face_bc;
    a.tiles = d.tiles;
    a.fscale = fp32 ? (const void *)d.fscalef : (const void *)d.fscale;
    a.mb = fp32 ? (const void *)d.mb32 : (const void *)d.mb64;
    a.mb1 = fp32 ? (const void *)d.mb1_32 : (const void *)d.mb1_64;
    for (int ax = 0; ax < 3; ++ax) a.xi[ax] = fp32 ? (const void *)d.xi32[ax] : (const void *)d.xi64[ax];
    int omax = 0;
    for (int o = 0; o < 8; ++o) omax = g.osize[o] > omax ? g.osize[o] : omax;
    int nvb = (omax + bs - 1) / bs;
    bool dia = g.species == 1;
    bool rfn = g.inv_dt != 0.0;
    for (int p = 0; p < nplane; ++p) {
        int off = plane_off[p], n = plane_cnt[p];
        if (n == 0) continue;
        if (fp32) {
            if (tx == 4 && ty == 4) sweep_plane<float, 4, 4>(a, dia, rfn, tz, off, n, nvb, bs, s);
            else if (tx == 8 && ty == 8) sweep_plane<float, 8, 8>(a, dia, rfn, tz, off, n, nvb, bs, s);
            else if (tx == 16 && ty == 8) sweep_plane<float, 16, 8>(a, dia, rfn, tz, off, n, nvb, bs, s);
            else return hipErrorInvalidValue;
        } else {
            if (tx == 4 && ty == 4) sweep_plane<double, 4, 4>(a, dia, rfn, tz, off, n, nvb, bs, s);
            else if (tx == 8 && ty == 4) sweep_plane<double, 8, 4>(a, dia, rfn, tz, off, n, nvb, bs, s);
            else if (tx == 8 && ty == 8) sweep_plane<double, 8, 8>(a, dia, rfn, tz, off, n, nvb, bs, s);
            else return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

}  // namespace gsis

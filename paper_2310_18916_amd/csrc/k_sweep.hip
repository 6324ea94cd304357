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
// thread, node-minor VDF layout, so every access is coalesced).  The tile is
// walked slab by slab (TX x TY cells at one z); a slab is fully unrolled, its
// values live in a register plane that is also the z-upwind input of the next
// slab, and cells on one slab diagonal are independent, which gives the
// scheduler instruction-level parallelism.  Nothing on the dependency chain
// waits for memory: the per-cell parameters and neighbour codes of the next
// slab are loaded cooperatively into LDS (double buffered, one barrier per
// slab), and the tile's inflow faces -- read from the VDF, which the upwind
// tile already holds in place, or the boundary values -- are prefetched into
// registers one slab ahead.  The reference distribution is evaluated on the
// fly from the per-cell parameters (FP32 copies on the FP32 path), one
// exponential per Maxwellian shape.  Every cell's update has a fixed operand
// order, so the result is bitwise independent of the tile shape and of the
// schedule.
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

// Value entering a cell through one upwind face: the neighbour's f^{n+1/2}
// (already final: the upwind tile ran in an earlier launch) or the boundary
// value rho_b M_b(xi) of the face.
template <typename T>
__device__ __forceinline__ T inflow(const SweepArgs &A, const T *f, const T *mbt, int nb, size_t node)
{
    const size_t nv = (size_t)A.g.nv;
    if (nb >= 0) return f[(size_t)nb * nv + node];
    const int fc = -nb - 1;
    return ((const T *)A.fscale)[fc] * mbt[(size_t)A.face_bc[fc] * nv + node];
}

template <typename T, int TX, int TY, bool DIA, bool RFN>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs A, int TZ, int plane_off, int nvb)
{
    constexpr int NPL = DIA ? 36 : 16;            // parameters per cell kept in LDS
    constexpr int NC = TX * TY;                   // cells per slab
    __shared__ T spar[2][NC * NPL];
    __shared__ int4 sinfo[2][NC];                 // fluid flag, upwind neighbour codes x, y, z

    const Geo &g = A.g;
    const int b = blockIdx.x;
    const int vb = b % nvb;
    const int o = (b / nvb) & 7;
    const int t = b / (nvb * 8);
    const int l = vb * blockDim.x + threadIdx.x;
    const bool active = l < g.osize[o];           // inactive threads still join loads and barriers
    const int packed = A.tiles[plane_off + t];
    const int tx = packed & 0x3ff, ty = (packed >> 10) & 0x3ff, tz = (packed >> 20) & 0x3ff;
    const int sx = o & 1, sy = (o >> 1) & 1, sz = (o >> 2) & 1;
    const int dxu = sx, dyu = 2 + sy, dzu = 4 + sz;   // upwind faces
    const int i0 = tx * TX, j0 = ty * TY, k0 = tz * TZ;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const size_t nv = (size_t)g.nv;

    T xix = T(0), xiy = T(0), xiz = T(0);
    size_t node = 0;
    if (active) {
        int kxn, kyn, kzn;
        node_of(g, o, l, kxn, kyn, kzn);
        xix = ((const T *)A.xi[0])[kxn];
        xiy = ((const T *)A.xi[1])[kyn];
        xiz = ((const T *)A.xi[2])[kzn];
        node = (size_t)g.obase[o] + l;
    }
    const T ax = fabs(xix) * (T)g.invh[0];
    const T ay = fabs(xiy) * (T)g.invh[1];
    const T az = fabs(xiz) * (T)g.invh[2];
    const T idt = (T)g.inv_dt;
    const T den0 = idt + ax + ay + az;
    T *f0 = (T *)A.f0;
    T *f1 = (T *)A.f1;
    const T *par = (const T *)A.par;
    const T *mb = (const T *)A.mb;
    const T *mb1 = (const T *)A.mb1;

    auto cell_at = [&](int kx, int ky, int kz) -> int {   // -1 outside the domain
        const int ii = i0 + kx, jj = j0 + ky, kk = k0 + kz;
        if (ii >= nx || jj >= ny || kk >= nz) return -1;
        const int i = sx ? nx - 1 - ii : ii, j = sy ? ny - 1 - jj : jj, k = sz ? nz - 1 - kk : kk;
        return i + nx * (j + ny * k);
    };
    // cooperative load of one slab's per-cell data into LDS buffer buf
    auto load_meta = [&](int kz, int buf) {
        for (int e = threadIdx.x; e < NC; e += blockDim.x) {
            const int c = cell_at(e % TX, e / TX, kz);
            int4 inf = make_int4(0, -1, -1, -1);
            if (c >= 0 && A.cflag[c]) {
                const int *nbc = A.nbr + (size_t)c * 6;
                inf = make_int4(1, nbc[dxu], nbc[dyu], nbc[dzu]);
            }
            sinfo[buf][e] = inf;
        }
        for (int e = threadIdx.x; e < NC * NPL; e += blockDim.x) {
            const int cc = e / NPL, k = e % NPL;
            const int c = cell_at(cc % TX, cc / TX, kz);
            spar[buf][e] = (c >= 0 && k < NPAR) ? par[(size_t)c * NPAR + k] : T(0);
        }
    };
    // inflow of the tile's x (rows) and y (columns) faces for slab kz
    auto load_xy = [&](int kz, T *xin0, T *xin1, T *yin0, T *yin1) {
#pragma unroll
        for (int ky = 0; ky < TY; ++ky) {
            xin0[ky] = T(0);
            if (DIA) xin1[ky] = T(0);
            const int c = cell_at(0, ky, kz);
            if (active && c >= 0 && A.cflag[c]) {
                const int nb = A.nbr[(size_t)c * 6 + dxu];
                xin0[ky] = inflow<T>(A, f0, mb, nb, node);
                if (DIA) xin1[ky] = inflow<T>(A, f1, mb1, nb, node);
            }
        }
#pragma unroll
        for (int kx = 0; kx < TX; ++kx) {
            yin0[kx] = T(0);
            if (DIA) yin1[kx] = T(0);
            const int c = cell_at(kx, 0, kz);
            if (active && c >= 0 && A.cflag[c]) {
                const int nb = A.nbr[(size_t)c * 6 + dyu];
                yin0[kx] = inflow<T>(A, f0, mb, nb, node);
                if (DIA) yin1[kx] = inflow<T>(A, f1, mb1, nb, node);
            }
        }
    };

    T pl0[TY][TX], pl1[TY][TX];                 // z-upwind plane, then the slab just computed
    T xin0[TY], xin1[TY], yin0[TX], yin1[TX];   // inflow faces of the current slab
    T xnx0[TY], xnx1[TY], ynx0[TX], ynx1[TX];   // ... and of the next slab

    load_meta(0, 0);
#pragma unroll
    for (int ky = 0; ky < TY; ++ky)
#pragma unroll
        for (int kx = 0; kx < TX; ++kx) {
            pl0[ky][kx] = T(0);
            pl1[ky][kx] = T(0);
            const int c = cell_at(kx, ky, 0);
            if (active && c >= 0 && A.cflag[c]) {
                const int nb = A.nbr[(size_t)c * 6 + dzu];
                pl0[ky][kx] = inflow<T>(A, f0, mb, nb, node);
                if (DIA) pl1[ky][kx] = inflow<T>(A, f1, mb1, nb, node);
            }
        }
    load_xy(0, xin0, xin1, yin0, yin1);
    __syncthreads();

    for (int kz = 0; kz < TZ; ++kz) {
        if (k0 + kz >= nz) break;                 // uniform over the block
        const int buf = kz & 1;
        const bool more = kz + 1 < TZ && k0 + kz + 1 < nz;
        if (more) {
            load_meta(kz + 1, buf ^ 1);
            load_xy(kz + 1, xnx0, xnx1, ynx0, ynx1);
        }
        if (active) {
#pragma unroll
            for (int ky = 0; ky < TY; ++ky) {
#pragma unroll
                for (int kx = 0; kx < TX; ++kx) {
                    const int e = ky * TX + kx;
                    const int4 inf = sinfo[buf][e];
                    if (!__builtin_amdgcn_readfirstlane(inf.x)) continue;
                    const int cell = cell_at(kx, ky, kz);
                    const int nbx = __builtin_amdgcn_readfirstlane(inf.y);
                    const int nby = __builtin_amdgcn_readfirstlane(inf.z);
                    const int nbz = __builtin_amdgcn_readfirstlane(inf.w);
                    const T *p = &spar[buf][e * NPL];
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
                    T F0, F1 = T(0);
                    // x upwind: the row's inflow, the cell just computed, or a solid neighbour's wall
                    if (kx == 0) { F0 = xin0[ky]; if (DIA) F1 = xin1[ky]; }
                    else if (nbx >= 0) { F0 = pl0[ky][kx - 1]; if (DIA) F1 = pl1[ky][kx - 1]; }
                    else { F0 = inflow<T>(A, f0, mb, nbx, node); if (DIA) F1 = inflow<T>(A, f1, mb1, nbx, node); }
                    num0 += ax * F0;
                    if (DIA) num1 += ax * F1;
                    if (ky == 0) { F0 = yin0[kx]; if (DIA) F1 = yin1[kx]; }
                    else if (nby >= 0) { F0 = pl0[ky - 1][kx]; if (DIA) F1 = pl1[ky - 1][kx]; }
                    else { F0 = inflow<T>(A, f0, mb, nby, node); if (DIA) F1 = inflow<T>(A, f1, mb1, nby, node); }
                    num0 += ay * F0;
                    if (DIA) num1 += ay * F1;
                    if (kz == 0 || nbz >= 0) { F0 = pl0[ky][kx]; if (DIA) F1 = pl1[ky][kx]; }
                    else { F0 = inflow<T>(A, f0, mb, nbz, node); if (DIA) F1 = inflow<T>(A, f1, mb1, nbz, node); }
                    num0 += az * F0;
                    if (DIA) num1 += az * F1;
                    const T den = den0 + invtau;
                    const T v0 = Arith<T>::div(num0, den);
                    f0[at] = v0;
                    pl0[ky][kx] = v0;
                    if (DIA) {
                        const T v1 = Arith<T>::div(num1, den);
                        f1[at] = v1;
                        pl1[ky][kx] = v1;
                    }
                }
            }
        }
        __syncthreads();
        if (more) {
#pragma unroll
            for (int ky = 0; ky < TY; ++ky) { xin0[ky] = xnx0[ky]; if (DIA) xin1[ky] = xnx1[ky]; }
#pragma unroll
            for (int kx = 0; kx < TX; ++kx) { yin0[kx] = ynx0[kx]; if (DIA) yin1[kx] = ynx1[kx]; }
        }
    }
}

// ------------------------------------------------------------------ launches
struct Shape { int tx, ty; };
// compiled (tx, ty) per precision; tz is a run-time loop length.  The slab is
// held in registers, so the diatomic gas (two planes) uses the small shapes.
static const Shape kShapes32[] = {{4, 4}, {8, 4}, {8, 8}};
static const Shape kShapes64[] = {{4, 4}, {8, 4}};

template <typename T, int TX, int TY>
static void sweep_plane(const SweepArgs &a, bool dia, bool rfn, int tz, int off, int ntile, int nvb, int bs,
                        hipStream_t s)
{
    constexpr bool kDia = TX * TY <= 32;   // two register planes only for the small slabs
    const size_t shm = 0;
    dim3 grid((unsigned)(ntile * 8 * nvb));
    if (dia) {
        if constexpr (kDia) {
            if (rfn) hipLaunchKernelGGL((k_sweep<T, TX, TY, true, true>), grid, dim3(bs), shm, s, a, tz, off, nvb);
            else hipLaunchKernelGGL((k_sweep<T, TX, TY, true, false>), grid, dim3(bs), shm, s, a, tz, off, nvb);
        }
    } else {
        if (rfn) hipLaunchKernelGGL((k_sweep<T, TX, TY, false, true>), grid, dim3(bs), shm, s, a, tz, off, nvb);
        else hipLaunchKernelGGL((k_sweep<T, TX, TY, false, false>), grid, dim3(bs), shm, s, a, tz, off, nvb);
    }
}

bool sweep_shape_supported(bool fp32, bool dia, int tx, int ty)
{
    if (dia && tx * ty > 32) return false;
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
            else if (tx == 8 && ty == 4) sweep_plane<float, 8, 4>(a, dia, rfn, tz, off, n, nvb, bs, s);
            else if (tx == 8 && ty == 8 && !dia) sweep_plane<float, 8, 8>(a, dia, rfn, tz, off, n, nvb, bs, s);
            else return hipErrorInvalidValue;
        } else {
            if (tx == 4 && ty == 4) sweep_plane<double, 4, 4>(a, dia, rfn, tz, off, n, nvb, bs, s);
            else if (tx == 8 && ty == 4) sweep_plane<double, 8, 4>(a, dia, rfn, tz, off, n, nvb, bs, s);
            else return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

}  // namespace gsis

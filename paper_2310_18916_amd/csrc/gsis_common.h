// Internal definitions shared by the libgsis kernels and the host runtime.
// Not part of the public ABI (see include/gsis.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsis {

constexpr int NRS = 17;    // raw moments stored per (cell, octant):
                           // 1, x, y, z, xx, yy, zz, xy, xz, yz, x|xi|^2, y|xi|^2, z|xi|^2 on f0,
                           // then 1, x, y, z on f1 (diatomic)
constexpr int NMOM = 18;   // central moments per cell (public order, diatomic tail)
constexpr int NPAR = 36;   // sweep parameters per cell
constexpr int NBC = 7;     // 6 box faces + solid surface
constexpr int NCORR = 12;  // pending GSIS correction per cell: new (rho,u,Tt,Tr), old (rho,u,Tt,Tr)
constexpr int NSNAP = 5;   // residual snapshot per cell: rho, u, Tt
constexpr double PI = 3.14159265358979323846;
constexpr int LSUM_SHAPE = 20;        // node list: Gram entries (15) and Shakhov moments (5) of one shape
constexpr int LSUM = 2 * LSUM_SHAPE;  // per cell: the Tt shape, then the T shape (diatomic)
constexpr int UMAXORI = 32;   // unstructured mesh: distinct face orientations (axes included)
constexpr int UMAXF = 16;     // unstructured mesh: faces per cell

// Geometry, velocity grid and gas constants, passed to kernels by value.
//
// Velocity octant o = sx + 2 sy + 4 sz with s_a = 1 when xi_a < 0 (a node with
// xi_a = 0 belongs to the positive half); the VDF of a cell is the 8 octants
// back to back.  Tensor grid (vlist = 0): along axis a the negative half is
// nodes [0, k0[a]) and the positive half [k0[a], n1[a]), and inside an octant
// the nodes are ordered x fastest.  Node list (vlist = 1, a refined or
// unstructured velocity mesh): an octant holds its nodes in the caller's
// order, n1 and k0 are 0 and on[o] = (osize[o], 1, 1).
struct Geo {
    int nx, ny, nz, ncell;
    double h[3], invh[3];
    int n1[3], k0[3];
    int nv;
    int vlist;
    int on[8][3];
    int osize[8];
    int obase[8];
    int species;
    double delta, omega, dr, Zr, A[4];
    double inv_dt;
    // explicit interface values of the kinetic update: order 1 (upwind) or 2
    // (limited least-squares reconstruction); (K h)^3 of the Venkatakrishnan
    // threshold (times the square of the stencil's largest |f| at each point)
    // and whether the limiter is on
    int order, limited;
    double venk_e2;
    double rs_scale;   // factor of the sweep's per-point term: inv_dt (order 1) or 1 (order 2)
    int conservative;
    double macro_cfl;
    int nface, nfluid;
    double kt, kr, gam, Cd;   // macroscopic transport constants
    double hmin;
    int fp32;      // VDF precision
    // unstructured spatial mesh (umesh = 1; nx = ncell, ny = nz = 1): ucls
    // velocity classes (the nodes whose signs of xi . n_k agree for every face
    // orientation n_k of the mesh, so that they share one upwind order), unbf
    // boundary faces, nori orientations
    int umesh, ucls, unbf, nori;
    int umaxcnt;   // nodes of the largest class
    int umaxf;     // faces of the cell with the most
    int unface;    // faces of the mesh
    int ucen;      // 1: centroids given (the macroscopic correction runs)
    double uhmin;  // smallest face distance h of the macroscopic pseudo time step
    // macroscopic boundary flux of the correction: 0 the Maxwellian's change,
    // 1 the Grad-13 distributions' change
    int wall_flux;
};

struct BcInfo {
    int kind[NBC];
    double u[NBC][3], T[NBC], rho[NBC];
};

// Device buffers, carved out of the caller's workspace.
// The global pseudo-time diagonal D* = max_i D_i is gathered by atomic max
// into DSLOT partial slots on separate cache lines (block b uses slot b mod
// DSLOT), so the atomics of different blocks do not queue on one address;
// readers take the max of the DSLOT partials.
constexpr int DSLOT = 64, DSTRIDE = 16;

struct Dev {
    void *f0, *f1;     // [ncell + 1][nv]: row ncell is the sink of the sweep's stores for dead cells
    // per-point term of the sweep's right-hand side, [ncell + 1][nv]: f0/f1
    // themselves (order 1, times inv_dt), or ho0/ho1 (order 2)
    void *rs0, *rs1;
    void *ho0, *ho1;   // order 2: inv_dt f^n - (second-order - first-order flux divergence), [ncell + 1][nv]
    void *lim0, *lim1; // order 2: Venkatakrishnan limiter per point, [ncell][nv]
    double *mom8;      // [ncell][8][NRS]
    double *cm;        // [ncell][NMOM]
    double *par;       // [ncell][NPAR]
    float *parf;       // [ncell][NPAR]
    int *cflag;        // [ncell] 1 = fluid
    int *nbr;          // [6][ncell]: neighbour cell, or -(face + 1)
    int *face_cell, *face_dir, *face_bc;   // [nface]
    double *fscale;    // [nface] density scale of the incoming half
    float *fscalef;
    double *cfs64;     // [ncell][6] the same scale by (cell, face direction), for the sweep
    float *cfs32;
    double *lsum;      // node list: [ncell][LSUM] shape sums of the relaxation parameters (else null)
    double *nt64;      // [nv][4] every node in the internal order: xi_x, xi_y, xi_z, weight
    float *nt32;       // [nv][4] the same in FP32
    double *xi64[3];   // per-axis nodes (tensor grid)
    float *xi32[3];
    double *w64[3];    // per-axis trapezoid weights
    double *xtab;      // [n1x][4]: w, w xi, w xi^2, w xi^3 along x
    double *ytab;      // [n1y][2]: w, xi
    double *ztab;      // [n1z][2]
    double *mb64, *mb1_64;   // [NBC][nv] boundary Maxwellian M(1,u_b,T_b), and (dr/2) T_b times it
    float *mb32, *mb1_32;
    double *inpsi;     // [NBC][6][6] incoming half-range psi-moments of M(1,u_b,T_b)
    int *perm;         // [nv] internal node -> canonical node
    int *tiles;        // sweep tile list grouped by plane
    int *plane_off;    // [nplane] first tile of each plane in tiles
    int *tent;         // [8 * tiles] (tile in plane << 3 | octant) entries of a split sweep: plane p's
                       // entries start at 8 plane_off[p], those without solid cells first
    // unstructured spatial mesh (null otherwise).  Face entries of every cell,
    // cell i's from the first face entry given with its sweep entries: ucf_nb
    // the cell on the other side, or -1 - b for boundary face b; ucf_meta = k |
    // s << 5 | slot << 6 with n_k the face's orientation, s = 1 when the
    // normal out of the cell is -n_k, and the boundary slot; ucf_g* [4] =
    // (S / V_i, unit normal out of the cell).  Classes ucls[c] = (sign mask:
    // bit k set when xi . n_k >= 0, first position in a VDF row, node count,
    // 0); ulev the sweep entries level after level, (cell << 8 | class, first
    // face entry << 5 | face count); boundary face b: its cell, slot, unit
    // normal out of the cell ([4] per face) and incoming density scale.
    double *uvol;      // [ncell] cell volumes (residual weights)
    int *ucf_nb, *ucf_meta;
    double *ucf_g64;
    float *ucf_g32;
    int4 *ucls;
    int2 *ulev;
    int *ubf_cell, *ubf_slot;
    double *ubf_n;
    double *ubf_s64;
    float *ubf_s32;
    // macroscopic correction on the mesh (centroids given): per face entry the
    // least-squares weights [3] of the neighbour across (0 on the boundary) and
    // the face (f << 1 | 1 when the cell is the face's neighbour); per face
    // (owner, neighbour or -1 - boundary face) and (S, n, h, |d|, d/|d|) [9];
    // the kinetic flux [6], its fixed part [6] and the iterate's flux and Gamma
    // [7]; per boundary face the incoming half-range psi-moments of its
    // boundary Maxwellian [6]
    double *ucf_lsq;
    int *ucf_face;
    int *ucf_first;    // [ncell + 1] first face entry of every cell
    int *ubf_face;     // [unbf] the face of every boundary face
    int *uf_cell;
    double *uf_geo, *uFk, *ufix, *uFf, *ubin;
    double *ubsq, *ubhot;   // Grad-13 wall flux: per boundary face [12][unbf] the stress of the iterate, HoT_c
    double *corr;      // [ncell][NCORR]
    double *snap;      // [ncell][NSNAP]
    // macroscopic solve, all structures of arrays [field][ncell] ([field][nface]
    // for fbfix, Fb): W (double buffered), prims P, velocity gradient,
    // high-order terms of the three + faces (six flux components each),
    // residual R
    double *W, *W2, *P, *grad, *hot, *R, *Dc, *Src, *fbfix, *Fb, *Gb;
    double *ghot;      // [12][nface] Grad-13 wall flux: the face cell's HoT_c (sigma 6, q 3, qr 3)
    double *red;       // reduction scratch
    unsigned long long *dmax;   // [2][DSLOT] partial maxima, one per 128-byte line (DSTRIDE words apart),
                                // bit patterns of positive doubles
    int *errflag;
    // residual history of a batch (nullptr for a context on its own):
    // hist[(iteration % hist_cap) * hist_ncase + hist_index][6], iteration = *hist_ctr
    double *hist;
    int *hist_ctr;
    int hist_index, hist_ncase, hist_cap;
};

// One case as the kernels of a GSIS iteration see it, resident in device
// memory, so that one launch can cover many independent cases.
struct Case {
    Geo g;
    BcInfo bc;
    Dev d;
    int tz;    // sweep tile depth
    int nvb;   // sweep blocks per octant (node runs of one block size)
};

// The blocks of a launch: map[b] = (case, block within that case), or, with
// map == nullptr, every block belongs to the first case of the table.
struct Span {
    const Case *cases;
    const int2 *map;
};

// Kernels take the span as two arguments.  The case table is read-only while
// kernels run, so it is read through the constant address space: its fields
// load through the scalar unit and, like kernel arguments, may be reloaded
// instead of being held in registers.
#define GSIS_SPAN_ARGS const gsis::Case *__restrict__ span_cases, const int2 *__restrict__ span_map
#define GSIS_SPAN(sp) (sp).cases, (sp).map
#define GSIS_CONST_AS __attribute__((address_space(4)))
// Buffers of a case are global memory; hot kernels keep their pointers in the
// global address space so that accesses use scalar base + vector offset.
#define GSIS_GLOBAL_AS __attribute__((address_space(1)))
template <class T> using gptr = GSIS_GLOBAL_AS T *;
// Read-only data every lane of a wave reads at the same index: the constant
// address space, so the reads go through the scalar unit.
template <class T> using cptr = const GSIS_CONST_AS T *;

// ------------------------------------------------------------ device helpers
// (case, block within the case) of the calling block; uniform over the block
__device__ __forceinline__ const Case &case_of(const Case *cases, const int2 *map, int &blk)
{
    int ci = 0;
    blk = (int)blockIdx.x;
    if (map) {
        const GSIS_CONST_AS int *m = (const GSIS_CONST_AS int *)(map + blockIdx.x);
        ci = m[0];
        blk = m[1];
    }
    return (const Case &)*(const GSIS_CONST_AS Case *)(cases + ci);
}

// e^x for |x| < 708: x = n ln2 + r with n = rint(x / ln2) and |r| <= ln2 / 2,
// the Cody-Waite two-part ln2 (the high part has 32 significant bits, so
// n ln2_hi is exact) keeping r exact to rounding; e^r by its Taylor
// polynomial to r^12 (truncation below 2e-16 relative on that interval),
// evaluated by Horner; 2^n through the exponent.
__device__ __forceinline__ double exp_core(double x)
{
    const double n = rint(x * 1.4426950408889634074);
    double r = fma(n, -6.93147180369123816490e-01, x);
    r = fma(n, -1.90821492927058770002e-10, r);
    double p = 1.0 / 479001600.0;
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)n);
}

// x^y for a normal x > 0 and moderate y (|y ln x| < 708), as e^{y ln x}:
// x = m 2^e with m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s) with
// s = (m - 1) / (m + 1), |s| < 0.172, by the odd series of atanh to s^23
// (truncation below 1e-18 relative), e ln2 in the two parts of exp_core.
// Within 8 ulp of the exact power for x in [1e-3, 1e3].
__device__ __forceinline__ double pow_pos(double x, double y)
{
    int e;
    double m = frexp(x, &e);
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0), s2 = s * s;
    double p = 1.0 / 23.0;
    p = fma(p, s2, 1.0 / 21.0);
    p = fma(p, s2, 1.0 / 19.0);
    p = fma(p, s2, 1.0 / 17.0);
    p = fma(p, s2, 1.0 / 15.0);
    p = fma(p, s2, 1.0 / 13.0);
    p = fma(p, s2, 1.0 / 11.0);
    p = fma(p, s2, 1.0 / 9.0);
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    p = fma(p, s2, 1.0);
    const double de = (double)e;
    const double lx = fma(de, 6.93147180369123816490e-01, fma(de, 1.90821492927058770002e-10, 2.0 * s * p));
    return exp_core(y * lx);
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One halving step of a transposing wave reduction: lanes with bit M set keep
// the upper half of their H + H values, the others the lower half, and each
// adds its partner's copy of the half it keeps.
template <int M, int H, int N>
__device__ __forceinline__ void halve(double (&v)[N], int lane, int &base)
{
    const bool hi = (lane & M) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const double send = hi ? v[i] : v[i + H];
        const double keep = hi ? v[i + H] : v[i];
        v[i] = keep + __shfl_xor(send, M, 64);
    }
    if (hi) base += H;
}

// Sums N (16 or 32) values over the 64 lanes of a wave in a fixed order with
// about N shuffles instead of N * 6: afterwards every lane holds the total of
// value *idx, and each value is held by the 64 / N lanes that share idx.
template <int N>
__device__ __forceinline__ double wave_reduce_scatter(double (&v)[N], int lane, int *idx)
{
    static_assert(N == 16 || N == 32, "16 or 32 values");
    int base = 0;
    if (N == 32) halve<32, 16>(v, lane, base);
    if (N == 32) halve<16, 8>(v, lane, base); else halve<32, 8>(v, lane, base);
    if (N == 32) halve<8, 4>(v, lane, base); else halve<16, 4>(v, lane, base);
    if (N == 32) halve<4, 2>(v, lane, base); else halve<8, 2>(v, lane, base);
    if (N == 32) halve<2, 1>(v, lane, base); else halve<4, 1>(v, lane, base);
    double r = v[0];
    constexpr int rest = 64 / N;   // lanes that still hold partial sums of the same value
#pragma unroll
    for (int m = 1; m < rest; m <<= 1) r += __shfl_xor(r, m, 64);
    *idx = base;
    return r;
}

// Maxwellian rho (pi T)^{-3/2} exp(-|xi - u|^2 / T) in units of sqrt(2 R T0).
__device__ __forceinline__ double maxwell64(double rho, const double *u, double T, double x, double y, double z)
{
    double cx = x - u[0], cy = y - u[1], cz = z - u[2];
    return rho * pow(PI * T, -1.5) * exp(-(cx * cx + cy * cy + cz * cz) / T);
}

}  // namespace gsis

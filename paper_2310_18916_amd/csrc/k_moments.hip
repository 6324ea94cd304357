// Moment reduction of Eq. (getmoment).
//
// k_moments: raw moments of every (cell, velocity octant) about the origin,
// accumulated in FP64 whatever the VDF precision.  The tensor grid makes the
// contraction separable: the x-rows of an octant (contiguous in the
// octant-grouped layout) give the four sums sum_x w_x xi_x^p f (p = 0..3),
// which fold with the row's y/z weights into the 13 (+4 for f1) monomials.
// One block per cell, one wave per octant, so per-octant sums -- from which
// every half-range wall flux follows -- need only a wave reduction.  Every
// load instruction reads one contiguous stretch of the VDF: rows of up to 20
// FP64 (32 FP32) values are staged through the wave's LDS region, 32 (64)
// rows at a time, and read back one row per lane; longer FP64 rows are read
// with the lanes along the rows (each keeping its columns and x-weights).
//
// k_derive: central moments (rho, u, Tt, sigma, q, Tr, qr) of every cell from
// the octant sums.
//
// k_commit_correction: adds to the octant sums the discrete raw moments of
// M(W') - M(W) of Eq. (updatef), which factor into 1-D sums on the tensor grid,
// so the corrected state's moments are exact without touching the VDF.
//
// On a node list (a refined or unstructured velocity mesh, Sec. 3.1) nothing
// factors: k_moments_list and k_commit_correction_list sum over the nodes
// directly, one wave per (cells, octant).
#include "gsis_common.h"
#include "gsis_launch.h"

namespace gsis {

// loads of VW consecutive elements of a row (global memory), widened to FP64
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T, int VW> struct VecLoad;
template <> struct VecLoad<float, 1> { static __device__ void ld(gptr<const float> p, double *o) { o[0] = p[0]; } };
template <> struct VecLoad<float, 2> {
    static __device__ void ld(gptr<const float> p, double *o)
    {
        f32x2 v = *(gptr<const f32x2>)p;
        o[0] = v.x; o[1] = v.y;
    }
};
template <> struct VecLoad<float, 4> {
    static __device__ void ld(gptr<const float> p, double *o)
    {
        f32x4 v = *(gptr<const f32x4>)p;
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    }
};
template <> struct VecLoad<double, 1> { static __device__ void ld(gptr<const double> p, double *o) { o[0] = p[0]; } };
template <> struct VecLoad<double, 2> {
    static __device__ void ld(gptr<const double> p, double *o)
    {
        f64x2 v = *(gptr<const f64x2>)p;
        o[0] = v.x; o[1] = v.y;
    }
};

// y and z (weight, node) tables staged in LDS when an axis has at most TABMAX
// nodes: the fold reads them once per row, which as global loads would
// outnumber the VDF loads
constexpr int TABMAX = 256;

template <typename T, int VW, bool DIA>
__global__ __launch_bounds__(512) void k_moments(GSIS_SPAN_ARGS)
{
    __shared__ double sty[2 * TABMAX], stz[2 * TABMAX];
    // FP32 rows of 4k values staged through LDS (64 rows per wave at a time)
    constexpr bool STG = sizeof(T) == 4 && VW == 4;
    constexpr int SROW = 32;
    __shared__ __attribute__((aligned(16))) float stg[STG ? 8 * 64 * SROW : 4];
    // FP64 rows of up to 20 values staged 32 at a time, each in a slot of at most 44 words
    constexpr bool STG64 = sizeof(T) == 8 && VW == 2;
    __shared__ __attribute__((aligned(16))) float stg64[STG64 ? 8 * 32 * 44 : 4];
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const gptr<const T> f0 = (gptr<const T>)C.d.f0;
    const gptr<const T> f1 = (gptr<const T>)C.d.f1;
    const gptr<const int> cflag = (gptr<const int>)C.d.cflag;
    const gptr<const double> xtab = (gptr<const double>)C.d.xtab;
    const gptr<const double> ytab = (gptr<const double>)C.d.ytab;
    const gptr<const double> ztab = (gptr<const double>)C.d.ztab;
    const gptr<double> mom8 = (gptr<double>)C.d.mom8;
    const int cell = blk;
    const int o = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const gptr<double> out = mom8 + ((size_t)cell * 8 + o) * NRS;
    if (!cflag[cell]) {
        if (lane < NRS) out[lane] = 0.0;
        return;
    }
    const bool staged = g.n1[1] <= TABMAX && g.n1[2] <= TABMAX;   // uniform over the block
    if (staged) {
        for (int i = threadIdx.x; i < 2 * g.n1[1]; i += blockDim.x) sty[i] = ytab[i];
        for (int i = threadIdx.x; i < 2 * g.n1[2]; i += blockDim.x) stz[i] = ztab[i];
    }
    __syncthreads();
    const int nox = g.on[o][0], noy = g.on[o][1], noz = g.on[o][2];
    const int x0 = (o & 1) ? 0 : g.k0[0];
    const int y0 = (o & 2) ? 0 : g.k0[1];
    const int z0 = (o & 4) ? 0 : g.k0[2];
    const size_t base = (size_t)cell * g.nv + g.obase[o];
    const int nrow = noy * noz;
    constexpr bool ALONG = sizeof(T) == 8 && VW == 2;   // the faster mapping for this layout (measured)
    double acc[13];
#pragma unroll
    for (int k = 0; k < 13; ++k) acc[k] = 0.0;
    double acc1[4] = {0.0, 0.0, 0.0, 0.0};
    const float rcp_noy = 1.0f / (float)noy;   // exact row -> (ly, lz) split for rows < 2^16
    // fold the x-sums s_p = sum_x w_x x^p f of row r with its y/z weights
    auto fold = [&](int r, double s0, double s1, double s2, double s3, double t0, double t1) {
        const int lz = (int)(((float)r + 0.5f) * rcp_noy), ly = r - lz * noy;
        double wy, y, wz, z;
        if (staged) {
            wy = sty[2 * (y0 + ly)]; y = sty[2 * (y0 + ly) + 1];
            wz = stz[2 * (z0 + lz)]; z = stz[2 * (z0 + lz) + 1];
        } else {
            wy = ytab[2 * (y0 + ly)]; y = ytab[2 * (y0 + ly) + 1];
            wz = ztab[2 * (z0 + lz)]; z = ztab[2 * (z0 + lz) + 1];
        }
        const double W0 = wy * wz;
        const double Y1 = W0 * y, Z1 = W0 * z;
        const double Y2 = Y1 * y, Z2 = Z1 * z, YZ = Y1 * z;
        const double Y3 = Y2 * y, Z3 = Z2 * z, YZ2 = YZ * z, Y2Z = Y2 * z;
        acc[0] += W0 * s0;
        acc[1] += W0 * s1;
        acc[2] += Y1 * s0;
        acc[3] += Z1 * s0;
        acc[4] += W0 * s2;
        acc[5] += Y2 * s0;
        acc[6] += Z2 * s0;
        acc[7] += Y1 * s1;
        acc[8] += Z1 * s1;
        acc[9] += YZ * s0;
        acc[10] += W0 * s3 + (Y2 + Z2) * s1;   // x |xi|^2 = x^3 + x y^2 + x z^2
        acc[11] += Y1 * s2 + (Y3 + YZ2) * s0;  // y |xi|^2 = x^2 y + y^3 + y z^2
        acc[12] += Z1 * s2 + (Y2Z + Z3) * s0;  // z |xi|^2 = x^2 z + y^2 z + z^3
        if (DIA) {
            acc1[0] += W0 * t0;
            acc1[1] += W0 * t1;
            acc1[2] += Y1 * t0;
            acc1[3] += Z1 * t0;
        }
    };
    // Two mappings, chosen by measurement.  Row per lane: each lane owns an
    // x-row and reads it in chunks whose loads are issued together (the
    // x-weights are wave-uniform).  Along the rows (FP64 pairs): lpr lanes
    // cover a row with VW elements each, 64 / lpr rows per load instruction,
    // so every load reads one contiguous stretch of the octant; a lane keeps
    // its columns (x-weights in registers) and issues UN rows' loads first.
    const int lpr = nox / VW;
    if (STG64 && nox <= 20) {
        // FP64 rows of at most 20 values: 32 rows at a time staged through the
        // wave's LDS region, each row in a slot of W words, W/4 odd, so the
        // 16 lanes of a b128 pass read disjoint banks
        const int W0 = nox * 2, W = (W0 >> 2) & 1 ? W0 : W0 + 4;
        const int vpr = nox >> 1;                  // 16-byte vectors per row
        float *sw = stg64 + o * 32 * 44;
        typedef float f4 __attribute__((ext_vector_type(4)));
        auto stage = [&](gptr<const T> fq, int r0, int nr) {
            const int nvec = nr * vpr;
            const gptr<const f4> src = (gptr<const f4>)(fq + base + (size_t)r0 * nox);
            f4 tmp[10];
#pragma unroll
            for (int k = 0; k < 10; ++k)
                if (lane + 64 * k < nvec) tmp[k] = __builtin_nontemporal_load(src + lane + 64 * k);
#pragma unroll
            for (int k = 0; k < 10; ++k) {
                const int v = lane + 64 * k;
                if (v < nvec) {
                    const int r = v / vpr, c = v - r * vpr;
                    *(f4 *)(sw + r * W + 4 * c) = tmp[k];
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        auto done = [&]() {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        for (int r0 = 0; r0 < nrow; r0 += 32) {
            const int nr = nrow - r0 < 32 ? nrow - r0 : 32;
            double s0 = 0, s1 = 0, s2 = 0, s3 = 0, t0 = 0, t1 = 0;
            stage(f0, r0, nr);
            if (lane < nr) {
                const double *row = (const double *)(sw + lane * W);
                for (int c = 0; c < nox; c += 2) {
                    const double e[2] = {row[c], row[c + 1]};
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const gptr<const double> xt = xtab + (size_t)(x0 + c + q) * 4;
                        s0 += xt[0] * e[q];
                        s1 += xt[1] * e[q];
                        s2 += xt[2] * e[q];
                        s3 += xt[3] * e[q];
                    }
                }
            }
            done();
            if (DIA) {
                stage(f1, r0, nr);
                if (lane < nr) {
                    const double *row = (const double *)(sw + lane * W);
                    for (int c = 0; c < nox; c += 2) {
                        const double e[2] = {row[c], row[c + 1]};
#pragma unroll
                        for (int q = 0; q < 2; ++q) {
                            const gptr<const double> xt = xtab + (size_t)(x0 + c + q) * 4;
                            t0 += xt[0] * e[q];
                            t1 += xt[1] * e[q];
                        }
                    }
                }
                done();
            }
            if (lane < nr) fold(r0 + lane, s0, s1, s2, s3, t0, t1);
        }
    } else if (STG && nox <= SROW) {
        // FP32 rows of at most SROW values: 64 rows at a time are staged
        // through this wave's LDS region with coalesced 16-byte loads (the 64
        // rows are one contiguous stretch of the octant), then each lane reads
        // its own row from LDS (rows of 4k floats: conflict-free b128 reads).
        // f1 passes through the same region after f0.  Only the lanes of one
        // wave share a region, so a wave barrier orders its writes and reads.
        float *sw = stg + o * 64 * SROW;
        typedef float f4 __attribute__((ext_vector_type(4)));
        auto stage = [&](gptr<const T> fq, int r0, int nr) {
            const int nvec = (nr * nox) >> 2;
            const gptr<const f4> src = (gptr<const f4>)(fq + base + (size_t)r0 * nox);
            f4 tmp[SROW / 4];
#pragma unroll
            for (int k = 0; k < SROW / 4; ++k)
                if (lane + 64 * k < nvec) tmp[k] = __builtin_nontemporal_load(src + lane + 64 * k);
#pragma unroll
            for (int k = 0; k < SROW / 4; ++k)
                if (lane + 64 * k < nvec) ((f4 *)sw)[lane + 64 * k] = tmp[k];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        auto done = [&]() {   // every lane has read its row before the region is overwritten
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        for (int r0 = 0; r0 < nrow; r0 += 64) {
            const int nr = nrow - r0 < 64 ? nrow - r0 : 64;
            double s0 = 0, s1 = 0, s2 = 0, s3 = 0, t0 = 0, t1 = 0;
            stage(f0, r0, nr);
            if (lane < nr) {
                const f4 *row = (const f4 *)(sw + lane * nox);
                for (int c = 0; c < (nox >> 2); ++c) {
                    const f4 v = row[c];
                    const double e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const gptr<const double> xt = xtab + (size_t)(x0 + 4 * c + q) * 4;
                        s0 += xt[0] * e[q];
                        s1 += xt[1] * e[q];
                        s2 += xt[2] * e[q];
                        s3 += xt[3] * e[q];
                    }
                }
            }
            done();
            if (DIA) {
                stage(f1, r0, nr);
                if (lane < nr) {
                    const f4 *row = (const f4 *)(sw + lane * nox);
                    for (int c = 0; c < (nox >> 2); ++c) {
                        const f4 v = row[c];
                        const double e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const gptr<const double> xt = xtab + (size_t)(x0 + 4 * c + q) * 4;
                            t0 += xt[0] * e[q];
                            t1 += xt[1] * e[q];
                        }
                    }
                }
                done();
            }
            if (lane < nr) fold(r0 + lane, s0, s1, s2, s3, t0, t1);
        }
    } else if (!ALONG) {
        // one row per lane, read in chunks of CH vectors issued together
        constexpr int CH0 = (DIA ? 64 : 128) / (VW * (int)sizeof(T));
        constexpr int CH = CH0 < 16 ? CH0 : 16;
        for (int r = lane; r < nrow; r += 64) {
            const gptr<const T> row0 = f0 + base + (size_t)r * nox;
            const gptr<const T> row1 = DIA ? f1 + base + (size_t)r * nox : row0;
            double s0 = 0, s1 = 0, s2 = 0, s3 = 0, t0 = 0, t1 = 0;
            // a row is read in chunks of CH vectors whose loads are all issued
            // before any is used, so the lines of a row are fetched together
            for (int lx0 = 0; lx0 < nox; lx0 += CH * VW) {
                double v[CH][VW], v1[CH][VW];
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    if (lx0 + c * VW < nox) {
                        VecLoad<T, VW>::ld(row0 + lx0 + c * VW, v[c]);
                        if (DIA) VecLoad<T, VW>::ld(row1 + lx0 + c * VW, v1[c]);
                    }
                }
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    if (lx0 + c * VW >= nox) break;
#pragma unroll
                    for (int e = 0; e < VW; ++e) {
                        const gptr<const double> xt = xtab + (size_t)(x0 + lx0 + c * VW + e) * 4;
                        s0 += xt[0] * v[c][e];
                        s1 += xt[1] * v[c][e];
                        s2 += xt[2] * v[c][e];
                        s3 += xt[3] * v[c][e];
                        if (DIA) {
                            t0 += xt[0] * v1[c][e];
                            t1 += xt[1] * v1[c][e];
                        }
                    }
                }
            }
            fold(r, s0, s1, s2, s3, t0, t1);
        }
    } else if (lpr <= 64) {
        const int rpi = 64 / lpr;
        const int my_r = lane / lpr, my_c = lane - my_r * lpr;
        if (my_r < rpi) {
            double wx[VW][4];
#pragma unroll
            for (int e = 0; e < VW; ++e)
#pragma unroll
                for (int q = 0; q < 4; ++q) wx[e][q] = xtab[(size_t)(x0 + my_c * VW + e) * 4 + q];
            constexpr int UN0 = (DIA ? 64 : 128) / (VW * (int)sizeof(T));
            constexpr int UN = UN0 < 16 ? UN0 : 16;
            for (int rb = my_r; rb < nrow; rb += UN * rpi) {
                double v[UN][VW], v1[UN][VW];
#pragma unroll
                for (int u = 0; u < UN; ++u) {
                    const int r = rb + u * rpi;
                    if (r < nrow) {
                        VecLoad<T, VW>::ld(f0 + base + (size_t)r * nox + my_c * VW, v[u]);
                        if (DIA) VecLoad<T, VW>::ld(f1 + base + (size_t)r * nox + my_c * VW, v1[u]);
                    }
                }
#pragma unroll
                for (int u = 0; u < UN; ++u) {
                    const int r = rb + u * rpi;
                    if (r >= nrow) break;
                    double s0 = 0, s1 = 0, s2 = 0, s3 = 0, t0 = 0, t1 = 0;
#pragma unroll
                    for (int e = 0; e < VW; ++e) {
                        s0 += wx[e][0] * v[u][e];
                        s1 += wx[e][1] * v[u][e];
                        s2 += wx[e][2] * v[u][e];
                        s3 += wx[e][3] * v[u][e];
                        if (DIA) {
                            t0 += wx[e][0] * v1[u][e];
                            t1 += wx[e][1] * v1[u][e];
                        }
                    }
                    fold(r, s0, s1, s2, s3, t0, t1);
                }
            }
        }
    } else {
        // rows longer than 64 vectors: the lanes take column groups of each row
        for (int r = 0; r < nrow; ++r) {
            double s0 = 0, s1 = 0, s2 = 0, s3 = 0, t0 = 0, t1 = 0;
            for (int c = lane; c < lpr; c += 64) {
                double v[VW], v1[VW];
                VecLoad<T, VW>::ld(f0 + base + (size_t)r * nox + c * VW, v);
                if (DIA) VecLoad<T, VW>::ld(f1 + base + (size_t)r * nox + c * VW, v1);
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    const gptr<const double> xt = xtab + (size_t)(x0 + c * VW + e) * 4;
                    s0 += xt[0] * v[e];
                    s1 += xt[1] * v[e];
                    s2 += xt[2] * v[e];
                    s3 += xt[3] * v[e];
                    if (DIA) {
                        t0 += xt[0] * v1[e];
                        t1 += xt[1] * v1[e];
                    }
                }
            }
            fold(r, s0, s1, s2, s3, t0, t1);
        }
    }
    // transposing reduction: lane groups end with one of the NRS sums each
    constexpr int NR = DIA ? 32 : 16;
    double v[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) v[k] = k < 13 ? acc[k < 13 ? k : 0] : (DIA && k < NRS ? acc1[k < NRS ? k - 13 : 0] : 0.0);
    int idx;
    const double r = wave_reduce_scatter<NR>(v, lane, &idx);
    if ((lane & (64 / NR - 1)) == 0 && idx < NRS) out[idx] = r;
    if (!DIA && lane == 0) out[NRS - 1] = 0.0;   // 13..15 come from the zero padding
}

// The 13 raw monomials of one node times its weight: 1, x, y, z, xx, yy, zz,
// xy, xz, yz, x|xi|^2, y|xi|^2, z|xi|^2.
__device__ __forceinline__ void node_monomials(const double *t, double m[13])
{
    const double x = t[0], y = t[1], z = t[2], w = t[3];
    m[0] = w;
    m[1] = w * x;
    m[2] = w * y;
    m[3] = w * z;
    m[4] = m[1] * x;
    m[5] = m[2] * y;
    m[6] = m[3] * z;
    m[7] = m[1] * y;
    m[8] = m[1] * z;
    m[9] = m[2] * z;
    const double s2 = x * x + y * y + z * z;
    m[10] = m[1] * s2;
    m[11] = m[2] * s2;
    m[12] = m[3] * s2;
}

// Writes the NRS sums of one (cell, octant) from the lanes' partial sums
// acc[0..12] (f0) and acc1[0..3] (f1), reduced over the wave in a fixed order.
template <bool DIA>
__device__ __forceinline__ void store_octant_sums(const double *acc, const double *acc1, int lane, gptr<double> out,
                                                  bool add)
{
    constexpr int NR = DIA ? 32 : 16;
    double v[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) v[k] = k < 13 ? acc[k < 13 ? k : 0] : (DIA && k < NRS ? acc1[k < NRS ? k - 13 : 0] : 0.0);
    int idx;
    const double r = wave_reduce_scatter<NR>(v, lane, &idx);
    if ((lane & (64 / NR - 1)) == 0 && idx < NRS) {
        if (add) out[idx] += r;
        else out[idx] = r;
    }
    if (!DIA && !add && lane == 0) out[NRS - 1] = 0.0;
}

// Node list: one wave (block) per octant of a group of CG consecutive cells.
// A lane takes the octant's nodes 64 apart, reads each node's (xi, w) once
// and applies its monomials to the node's value in every cell of the group,
// so the node table is read once per CG cells while each VDF load covers 64
// consecutive nodes of one cell.  Two nodes per lane and step, and the loads
// of all cells issued unconditionally (rows clamped to the last cell, a dead
// or missing cell's sums discarded at the end), keep 2 CG loads in flight.
template <typename T, bool DIA, int CG>
__global__ __launch_bounds__(64) void k_moments_list(GSIS_SPAN_ARGS)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const gptr<const int> cflag = (gptr<const int>)C.d.cflag;
    const gptr<const double> nt = (gptr<const double>)C.d.nt64;
    const gptr<double> mom8 = (gptr<double>)C.d.mom8;
    const int o = blk & 7;
    const int cell0 = (blk >> 3) * CG;
    const int lane = threadIdx.x;
    const int n = g.osize[o], ob = g.obase[o];
    const size_t nv = (size_t)g.nv;
    gptr<const T> r0[CG], r1[CG];
    bool live[CG];
#pragma unroll
    for (int c = 0; c < CG; ++c) {
        const int cc = min(cell0 + c, g.ncell - 1);
        live[c] = cell0 + c < g.ncell && cflag[cc];   // uniform over the wave
        r0[c] = (gptr<const T>)C.d.f0 + (size_t)cc * nv + ob;
        r1[c] = DIA ? (gptr<const T>)C.d.f1 + (size_t)cc * nv + ob : r0[c];
    }
    double acc[CG][13], acc1[CG][4];
#pragma unroll
    for (int c = 0; c < CG; ++c) {
#pragma unroll
        for (int k = 0; k < 13; ++k) acc[c][k] = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) acc1[c][k] = 0.0;
    }
    for (int l0 = 0; l0 < n; l0 += 128) {
        int li[2];
        double sc[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int l = l0 + h * 64 + lane;
            li[h] = min(l, n - 1);
            sc[h] = l < n ? 1.0 : 0.0;   // a repeated last node counts zero
        }
        T v[2][CG], v1[2][CG];
        double t[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int c = 0; c < CG; ++c) {
                v[h][c] = r0[c][li[h]];
                if (DIA) v1[h][c] = r1[c][li[h]];
            }
            const gptr<const double> tp = nt + 4 * ((size_t)ob + li[h]);
#pragma unroll
            for (int q = 0; q < 4; ++q) t[h][q] = tp[q];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            t[h][3] *= sc[h];
            double m[13];
            node_monomials(t[h], m);
#pragma unroll
            for (int c = 0; c < CG; ++c) {
                const double x = (double)v[h][c];
#pragma unroll
                for (int k = 0; k < 13; ++k) acc[c][k] += m[k] * x;
                if (DIA) {
                    const double x1 = (double)v1[h][c];
#pragma unroll
                    for (int k = 0; k < 4; ++k) acc1[c][k] += m[k] * x1;
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CG; ++c) {
        if (cell0 + c >= g.ncell) break;
        if (!live[c]) {
#pragma unroll
            for (int k = 0; k < 13; ++k) acc[c][k] = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) acc1[c][k] = 0.0;
        }
        store_octant_sums<DIA>(acc[c], acc1[c], lane, mom8 + ((size_t)(cell0 + c) * 8 + o) * NRS, false);
    }
}

// Central moments from the octant sums (octants added in a fixed order).
__global__ __launch_bounds__(256) void k_derive(GSIS_SPAN_ARGS)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    int cell = blk * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    double *out = d.cm + (size_t)cell * NMOM;
    if (!d.cflag[cell]) {
        for (int k = 0; k < NMOM; ++k) out[k] = __builtin_nan("");
        return;
    }
    double m[NRS];
    for (int k = 0; k < NRS; ++k) m[k] = 0.0;
    for (int o = 0; o < 8; ++o) {
        const double *mo = d.mom8 + ((size_t)cell * 8 + o) * NRS;
        for (int k = 0; k < NRS; ++k) m[k] += mo[k];
    }
    double rho = m[0];
    double u[3] = {m[1] / rho, m[2] / rho, m[3] / rho};
    // second raw moments as a matrix
    double M2[3][3] = {{m[4], m[7], m[8]}, {m[7], m[5], m[9]}, {m[8], m[9], m[6]}};
    double S[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) S[a][b] = M2[a][b] - rho * u[a] * u[b];
    double tr = S[0][0] + S[1][1] + S[2][2];
    double Tt = (2.0 / 3.0) * tr / rho;
    double tr2 = M2[0][0] + M2[1][1] + M2[2][2];
    double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    out[0] = rho;
    out[1] = u[0];
    out[2] = u[1];
    out[3] = u[2];
    out[4] = Tt;
    out[5] = 2.0 * (S[0][0] - tr / 3.0);
    out[6] = 2.0 * (S[1][1] - tr / 3.0);
    out[7] = 2.0 * (S[2][2] - tr / 3.0);
    out[8] = 2.0 * S[0][1];
    out[9] = 2.0 * S[0][2];
    out[10] = 2.0 * S[1][2];
    // q_a = sum c_a |c|^2 f = m3_a - 2 (M2 u)_a - u_a tr(M2) + 2 rho u_a |u|^2
    for (int a = 0; a < 3; ++a) {
        double m2u = M2[a][0] * u[0] + M2[a][1] * u[1] + M2[a][2] * u[2];
        out[11 + a] = m[10 + a] - 2.0 * m2u - u[a] * tr2 + 2.0 * rho * u[a] * u2;
    }
    if (g.species == 1) {
        double e1 = m[13];
        out[14] = 2.0 * e1 / (g.dr * rho);
        for (int a = 0; a < 3; ++a) out[15 + a] = m[14 + a] - u[a] * e1;
    } else {
        out[14] = out[15] = out[16] = out[17] = 0.0;
    }
    if (!(rho > 0.0) || !(Tt > 0.0)) atomicOr(d.errflag, 1);
}

// 1-D sums over the negative (h = 0) and positive (h = 1) halves of one axis:
// R[h][p] = sum_k w_k xi_k^p exp(-(xi_k - u)^2 / T), p = 0..3.
__device__ void half_sums(const double *xi, const double *w, int n, int k0, double u, double T, double R[2][4])
{
    for (int h = 0; h < 2; ++h)
        for (int p = 0; p < 4; ++p) R[h][p] = 0.0;
    for (int k = 0; k < n; ++k) {
        double x = xi[k], c = x - u;
        double e = w[k] * exp(-c * c / T);
        int h = k >= k0;
        R[h][0] += e;
        R[h][1] += e * x;
        R[h][2] += e * x * x;
        R[h][3] += e * x * x * x;
    }
}

// Raw octant moments (13 on f0, 4 on f1) of K * prod_a exp(-(xi_a-u_a)^2/T) given the
// half sums of each axis; f1 gets the factor h1.
__device__ void octant_monomials(const double X[4], const double Y[4], const double Z[4], double K, double h1,
                                 double *m)
{
    m[0] = K * X[0] * Y[0] * Z[0];
    m[1] = K * X[1] * Y[0] * Z[0];
    m[2] = K * X[0] * Y[1] * Z[0];
    m[3] = K * X[0] * Y[0] * Z[1];
    m[4] = K * X[2] * Y[0] * Z[0];
    m[5] = K * X[0] * Y[2] * Z[0];
    m[6] = K * X[0] * Y[0] * Z[2];
    m[7] = K * X[1] * Y[1] * Z[0];
    m[8] = K * X[1] * Y[0] * Z[1];
    m[9] = K * X[0] * Y[1] * Z[1];
    m[10] = K * (X[3] * Y[0] * Z[0] + X[1] * Y[2] * Z[0] + X[1] * Y[0] * Z[2]);
    m[11] = K * (X[2] * Y[1] * Z[0] + X[0] * Y[3] * Z[0] + X[0] * Y[1] * Z[2]);
    m[12] = K * (X[2] * Y[0] * Z[1] + X[0] * Y[2] * Z[1] + X[0] * Y[0] * Z[3]);
    m[13] = h1 * m[0];
    m[14] = h1 * m[1];
    m[15] = h1 * m[2];
    m[16] = h1 * m[3];
}

// Octant sums += moments of M(W') - M(W) (and (dr/2)[Tr' M(W') - Tr M(W)] on f1).
__global__ __launch_bounds__(128) void k_commit_correction(GSIS_SPAN_ARGS)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    int cell = blk * blockDim.x + threadIdx.x;
    if (cell >= g.ncell || !d.cflag[cell]) return;
    const double *c = d.corr + (size_t)cell * NCORR;
    double Rn[3][2][4], Ro[3][2][4];
    for (int a = 0; a < 3; ++a) {
        half_sums(d.xi64[a], d.w64[a], g.n1[a], g.k0[a], c[1 + a], c[4], Rn[a]);
        half_sums(d.xi64[a], d.w64[a], g.n1[a], g.k0[a], c[7 + a], c[10], Ro[a]);
    }
    double Kn = c[0] * pow(PI * c[4], -1.5), Ko = c[6] * pow(PI * c[10], -1.5);
    double hn = g.species == 1 ? 0.5 * g.dr * c[5] : 0.0;
    double ho = g.species == 1 ? 0.5 * g.dr * c[11] : 0.0;
    for (int o = 0; o < 8; ++o) {
        int hx = (o & 1) ? 0 : 1, hy = (o & 2) ? 0 : 1, hz = (o & 4) ? 0 : 1;
        double mn[NRS], mo[NRS];
        octant_monomials(Rn[0][hx], Rn[1][hy], Rn[2][hz], Kn, hn, mn);
        octant_monomials(Ro[0][hx], Ro[1][hy], Ro[2][hz], Ko, ho, mo);
        double *dst = d.mom8 + ((size_t)cell * 8 + o) * NRS;
        for (int k = 0; k < NRS; ++k) dst[k] += mn[k] - mo[k];
    }
}

// Node list: octant sums += moments of M(W') - M(W) (and (dr/2)[Tr' M(W') -
// Tr M(W)] on f1), one wave per octant of one cell, summed over the nodes.
__global__ __launch_bounds__(512) void k_commit_correction_list(GSIS_SPAN_ARGS)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const int cell = blk;
    const gptr<const int> cflag = (gptr<const int>)C.d.cflag;
    if (!cflag[cell]) return;   // uniform over the block
    const int o = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const gptr<const double> nt = (gptr<const double>)C.d.nt64;
    const gptr<const double> c = (gptr<const double>)C.d.corr + (size_t)cell * NCORR;
    const double pn = PI * c[4], po = PI * c[10];
    const double Kn = c[0] / (pn * sqrt(pn)), Ko = c[6] / (po * sqrt(po));
    const double itn = 1.0 / c[4], ito = 1.0 / c[10];
    const bool dia = g.species == 1;
    const double hn = dia ? 0.5 * g.dr * c[5] : 0.0, ho = dia ? 0.5 * g.dr * c[11] : 0.0;
    double acc[13], acc1[4];
#pragma unroll
    for (int k = 0; k < 13; ++k) acc[k] = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) acc1[k] = 0.0;
    const int n = g.osize[o], ob = g.obase[o];
    for (int l = lane; l < n; l += 64) {
        const size_t node = (size_t)ob + l;
        const double t[4] = {nt[4 * node], nt[4 * node + 1], nt[4 * node + 2], nt[4 * node + 3]};
        const double nx = t[0] - c[1], ny = t[1] - c[2], nz = t[2] - c[3];
        const double ox = t[0] - c[7], oy = t[1] - c[8], oz = t[2] - c[9];
        const double en = Kn * exp_core(fmax(-(nx * nx + ny * ny + nz * nz) * itn, -745.0));
        const double eo = Ko * exp_core(fmax(-(ox * ox + oy * oy + oz * oz) * ito, -745.0));
        const double d0 = en - eo, d1 = hn * en - ho * eo;
        double m[13];
        node_monomials(t, m);
#pragma unroll
        for (int k = 0; k < 13; ++k) acc[k] += m[k] * d0;
#pragma unroll
        for (int k = 0; k < 4; ++k) acc1[k] += m[k] * d1;
    }
    const gptr<double> out = (gptr<double>)C.d.mom8 + ((size_t)cell * 8 + o) * NRS;
    if (dia) store_octant_sums<true>(acc, acc1, lane, out, true);
    else store_octant_sums<false>(acc, acc1, lane, out, true);
}

// ------------------------------------------------------------------ launches
template <typename T, int VW>
static void moments_vw(const Target &t, int cls, hipStream_t s)
{
    const Span sp{t.cases, t.mom_map[cls]};
    const dim3 grid(t.mom_nblk[cls]);
    if (t.dia) hipLaunchKernelGGL((k_moments<T, VW, true>), grid, dim3(512), 0, s, GSIS_SPAN(sp));
    else hipLaunchKernelGGL((k_moments<T, VW, false>), grid, dim3(512), 0, s, GSIS_SPAN(sp));
}

// One launch per vector-width class present (a case's width follows its
// octant row lengths), so every case is reduced exactly as on its own.
// cells per block of the node-list moment kernel
template <bool DIA> constexpr int list_cg() { return DIA ? 2 : 4; }

template <typename T, bool DIA>
static void moments_list(const Target &t, hipStream_t s)
{
    constexpr int CG = list_cg<DIA>();
    const int ncell = t.host[0].g.ncell;
    hipLaunchKernelGGL((k_moments_list<T, DIA, CG>), dim3(8 * ((ncell + CG - 1) / CG)), dim3(64), 0, s,
                       GSIS_SPAN(t.span(K_CELL1)));
}

hipError_t launch_moments(const Target &t, hipStream_t s)
{
    if (t.vlist) {
        // one case (batches hold tensor grids only)
        if (t.fp32) { if (t.dia) moments_list<float, true>(t, s); else moments_list<float, false>(t, s); }
        else { if (t.dia) moments_list<double, true>(t, s); else moments_list<double, false>(t, s); }
        return hipGetLastError();
    }
    if (t.mom_nblk[0] > 0) {
        if (t.fp32) moments_vw<float, 1>(t, 0, s);
        else moments_vw<double, 1>(t, 0, s);
    }
    if (t.mom_nblk[1] > 0) {
        if (t.fp32) moments_vw<float, 2>(t, 1, s);
        else moments_vw<double, 2>(t, 1, s);
    }
    if (t.mom_nblk[2] > 0) {
        if (t.fp32) moments_vw<float, 4>(t, 2, s);
        else moments_vw<double, 2>(t, 2, s);   // FP64 rows load two at a time at most
    }
    return hipGetLastError();
}

hipError_t launch_derive(const Target &t, hipStream_t s)
{
    hipLaunchKernelGGL(k_derive, dim3(t.nblk[K_CELL256]), dim3(256), 0, s, GSIS_SPAN(t.span(K_CELL256)));
    return hipGetLastError();
}

hipError_t launch_commit_correction(const Target &t, hipStream_t s)
{
    if (t.vlist) {
        hipLaunchKernelGGL(k_commit_correction_list, dim3(t.host[0].g.ncell), dim3(512), 0, s,
                           GSIS_SPAN(t.span(K_CELL1)));
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_commit_correction, dim3(t.nblk[K_CELL128]), dim3(128), 0, s, GSIS_SPAN(t.span(K_CELL128)));
    return hipGetLastError();
}

}  // namespace gsis

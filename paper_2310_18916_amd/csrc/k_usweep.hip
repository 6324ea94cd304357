// The kinetic update of Sec. 3.2 on an unstructured spatial mesh, solved
// exactly.
//
// With first-order upwind interface values on both sides of Eq.
// (delta_equations), cell i of volume V_i with faces of area S_ij and unit
// normal n_ij (out of i) gets, for one velocity node,
//   f_i^{n+1/2} = [f_i^n / dt + g_i / tau_i + sum_{xi.n_ij < 0} a_ij F_ij]
//                 / (1/dt + 1/tau_i + sum_{xi.n_ij > 0} a_ij),
//   a_ij = |xi . n_ij| S_ij / V_i,
// F_ij the new value of neighbour j or the boundary value of the face.  The
// system of one node is lower triangular in the order of its upwind graph.
// The host groups the nodes into classes that agree on the sign of xi . n_k
// for every face orientation n_k of the mesh: the nodes of a class share one
// upwind graph, whose cells it sorts into levels (a cell's level is one more
// than the highest level upwind of it).  Launch L updates, for every class,
// the cells of that class's level L: one wave per (cell, class), a lane per
// node of the class, the nodes of a class contiguous in every VDF row (so
// every access is coalesced), the VDF updated in place.  Which faces bring a
// node in is read from the class's sign mask, the same for every lane of the
// wave, never from a recomputed sign, so a node can only read values its
// class's order has already written.  Each cell's faces are taken in a fixed
// order, so the result does not depend on the schedule.
#include "gsis.h"
#include "gsis_common.h"
#include "gsis_launch.h"
#include "gsis_sweep_math.h"

namespace gsis {

// Incoming density scale of every boundary face, from f^n of its cell: a
// diffuse wall gets rho_w = sum_{xi.n>0} w xi.n f0 / sum_{xi.n<0} w |xi.n| M_w
// (zero discrete mass flux through the wall), an inflow face its fixed
// density.  With a GSIS correction pending (committed to the moments, not yet
// to the stored VDF: a source-iteration pass never reads f^n otherwise) f^n
// is the stored row plus M(W^{n+1}) - M(W^{n+1/2}) of Eq. (updatef), formed
// here per node.  One wave per face, FP64 sums, lane partials combined by a
// fixed butterfly.
template <typename T>
__global__ __launch_bounds__(256) void k_uface_scale(GSIS_SPAN_ARGS, int pend)
{
    int b;
    const Case &C = case_of(span_cases, span_map, b);
    const Geo &g = C.g;
    const int bf = __builtin_amdgcn_readfirstlane(b * 4 + (int)(threadIdx.x >> 6));
    if (bf >= g.unbf) return;
    const int lane = threadIdx.x & 63;
    const int cell = C.d.ubf_cell[bf], slot = C.d.ubf_slot[bf];
    double scale = C.bc.rho[slot];
    if (C.bc.kind[slot] != GSIS_MAXWELL_INFLOW) {
        const double nx = C.d.ubf_n[4 * bf], ny = C.d.ubf_n[4 * bf + 1], nz = C.d.ubf_n[4 * bf + 2];
        const size_t nv = (size_t)g.nv;
        const T *f = (const T *)C.d.f0 + (size_t)cell * nv;
        const double *mb = C.d.mb64 + (size_t)slot * nv;
        const double *c = C.d.corr + (size_t)cell * NCORR;
        const double pn = PI * c[4], po = PI * c[10];
        const double an = c[0] / (pn * sqrt(pn)), ao = c[6] / (po * sqrt(po));
        const double itn = 1.0 / c[4], ito = 1.0 / c[10];
        double out = 0.0, in = 0.0;
        for (int pos = lane; pos < g.nv; pos += 64) {
            const double *t = C.d.nt64 + 4 * (size_t)pos;
            const double xn = t[0] * nx + t[1] * ny + t[2] * nz;
            if (xn > 0.0) {
                double fv = (double)f[pos];
                if (pend) {
                    const double ex = t[0] - c[1], ey = t[1] - c[2], ez = t[2] - c[3];
                    const double ox = t[0] - c[7], oy = t[1] - c[8], oz = t[2] - c[9];
                    fv += an * exp_core(fmax(-(ex * ex + ey * ey + ez * ez) * itn, -745.0)) -
                          ao * exp_core(fmax(-(ox * ox + oy * oy + oz * oz) * ito, -745.0));
                }
                out += t[3] * xn * fv;
            } else if (xn < 0.0) {
                in += t[3] * (-xn) * mb[pos];
            }
        }
        scale = wave_sum(out) / wave_sum(in);
    }
    if (lane == 0) {
        C.d.ubf_s64[bf] = scale;
        C.d.ubf_s32[bf] = (float)scale;
    }
}

// Sweep entries [e0, e1) of one level, one wave each: entry (cell << 8 |
// class, first face entry << 5 | face count).  The wave walks the class's
// nodes 64 at a time; the loads of the next 64 (inflow values and node
// velocities) are issued before the current 64 are computed, so a wave keeps
// two rounds of memory traffic in flight.  MAXF bounds the faces of a cell.
// FP32: eight waves per SIMD (measured 7% faster than the seven its scalar
// registers would allow), except the diatomic gas with more than 8 faces per
// cell, which would spill; FP64 keeps its registers (eight waves spill).
template <typename T, bool DIA, int MAXF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((sizeof(T) == 4 && !(DIA && MAXF > 8)) ? 8 : 1))) void k_usweep(GSIS_SPAN_ARGS, int e0, int e1)
{
#pragma clang fp contract(off)
    constexpr bool F32 = sizeof(T) == 4;
    constexpr int NP = DIA ? 34 : 14;   // sweep parameters the reference distribution reads
    int b;
    const Case &C = case_of(span_cases, span_map, b);
    const Geo &g = C.g;
    const int e = __builtin_amdgcn_readfirstlane(e0 + b * 4 + (int)(threadIdx.x >> 6));
    if (e >= e1) return;   // uniform over the wave
    const int lane = threadIdx.x & 63;
    const cptr<int> ent = (cptr<int>)(C.d.ulev + e);
    const int cell = ent[0] >> 8, cls = ent[0] & 255;
    const int fb = ent[1] >> 5, nf = ent[1] & 31;
    const cptr<int> cl = (cptr<int>)(C.d.ucls + cls);
    const unsigned mask = (unsigned)cl[0];
    const int pos0 = cl[1], cnt = cl[2];
    const cptr<T> par = (F32 ? (cptr<T>)C.d.parf : (cptr<T>)C.d.par) + (size_t)cell * NPAR;
    T p[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) p[k] = par[k];
    const cptr<int> cnb = (cptr<int>)C.d.ucf_nb + fb;
    const cptr<int> cmeta = (cptr<int>)C.d.ucf_meta + fb;
    const cptr<T> cgeo = (F32 ? (cptr<T>)C.d.ucf_g32 : (cptr<T>)C.d.ucf_g64) + 4 * (size_t)fb;
    const cptr<T> bsc = F32 ? (cptr<T>)C.d.ubf_s32 : (cptr<T>)C.d.ubf_s64;
    const gptr<const T> nt = F32 ? (gptr<const T>)C.d.nt32 : (gptr<const T>)C.d.nt64;
    const gptr<const T> mb = F32 ? (gptr<const T>)C.d.mb32 : (gptr<const T>)C.d.mb64;
    const gptr<const T> mb1 = F32 ? (gptr<const T>)C.d.mb1_32 : (gptr<const T>)C.d.mb1_64;
    const size_t nv = (size_t)g.nv;
    const gptr<T> f0 = (gptr<T>)C.d.f0, f1 = (gptr<T>)C.d.f1;
    const T idt = (T)g.inv_dt;
    const bool fdt = g.inv_dt != 0.0;
    const T invtau = DIA ? p[33] : p[13];

    // the faces of the cell: which bring the class's nodes in, from where, and
    // their (S / V, unit normal out of the cell)
    int src[MAXF];       // cell row of an interior inflow face, or -1 - boundary face
    int slot[MAXF];
    bool in[MAXF];
    T geo[MAXF][4];
#pragma unroll
    for (int j = 0; j < MAXF; ++j) {
        if (j < nf) {
            const int meta = cmeta[j];
            const bool flip = (meta >> 5) & 1;
            in[j] = (((mask >> (meta & 31)) & 1u) != 0) == flip;   // xi . n out of the cell < 0 for the class
            src[j] = cnb[j];
            slot[j] = (meta >> 6) & 7;
#pragma unroll
            for (int q = 0; q < 4; ++q) geo[j][q] = cgeo[4 * j + q];
        } else {
            in[j] = false;
            src[j] = 0;
            slot[j] = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) geo[j][q] = T(0);
        }
    }
    // the loads of one run of 64 nodes: velocities, inflow values, f^n of the cell (finite dt)
    struct Run { T x, y, z, o0, o1, F0[MAXF], F1[MAXF]; };
    auto load = [&](int l0, Run &r) {
        const int l = min(l0 + lane, cnt - 1);
        const size_t pos = (size_t)pos0 + l;
        r.x = nt[4 * pos];
        r.y = nt[4 * pos + 1];
        r.z = nt[4 * pos + 2];
#pragma unroll
        for (int j = 0; j < MAXF; ++j) {
            r.F0[j] = r.F1[j] = T(0);
            if (j < nf && in[j]) {
                if (src[j] >= 0) {
                    r.F0[j] = f0[(size_t)src[j] * nv + pos];
                    if (DIA) r.F1[j] = f1[(size_t)src[j] * nv + pos];
                } else {
                    const T sc = bsc[-1 - src[j]];
                    r.F0[j] = sc * mb[(size_t)slot[j] * nv + pos];
                    if (DIA) r.F1[j] = sc * mb1[(size_t)slot[j] * nv + pos];
                }
            }
        }
        r.o0 = r.o1 = T(0);
        if (fdt) {
            r.o0 = f0[(size_t)cell * nv + pos];
            if (DIA) r.o1 = f1[(size_t)cell * nv + pos];
        }
    };
    Run cur, nxt;
    load(0, cur);
    for (int l0 = 0; l0 < cnt; l0 += 64) {
        if (l0 + 64 < cnt) load(l0 + 64, nxt);   // uniform
        const T cx = cur.x - p[0], cy = cur.y - p[1], cz = cur.z - p[2];
        T num0, num1 = T(0);
        if (DIA) ref_dia<T>(p, cx, cy, cz, p[3], p[4], num0, num1);
        else num0 = ref_mono<T>(p, cx, cy, cz, p[3]);
        num0 = fma(idt, cur.o0, num0);
        if (DIA) num1 = fma(idt, cur.o1, num1);
        T den = idt + invtau;
#pragma unroll
        for (int j = 0; j < MAXF; ++j) {
            if (j < nf) {
                const T xn = fma(cur.z, geo[j][3], fma(cur.y, geo[j][2], cur.x * geo[j][1]));
                const T a = fabs(xn) * geo[j][0];
                if (in[j]) {
                    num0 = fma(a, cur.F0[j], num0);
                    if (DIA) num1 = fma(a, cur.F1[j], num1);
                } else {
                    den += a;
                }
            }
        }
        const int l = l0 + lane;
        if (l < cnt) {
            const size_t pos = (size_t)pos0 + l;
            f0[(size_t)cell * nv + pos] = Arith<T>::div(num0, den);
            if (DIA) f1[(size_t)cell * nv + pos] = Arith<T>::div(num1, den);
        }
        cur = nxt;
    }
}

hipError_t launch_uface_scale(const Target &t, int pending, hipStream_t s)
{
    const Geo &g = t.host->g;
    if (g.unbf == 0) return hipSuccess;
    const dim3 grid((g.unbf + 3) / 4);
    if (t.fp32) hipLaunchKernelGGL(k_uface_scale<float>, grid, dim3(256), 0, s, t.cases, nullptr, pending);
    else hipLaunchKernelGGL(k_uface_scale<double>, grid, dim3(256), 0, s, t.cases, nullptr, pending);
    return hipGetLastError();
}

hipError_t launch_usweep(const Target &t, const int *lev_off, int nlev, hipStream_t s)
{
    const int mf = t.host->g.umaxf;
    for (int L = 0; L < nlev; ++L) {
        const int e0 = lev_off[L], e1 = lev_off[L + 1];
        if (e1 <= e0) continue;
        const dim3 grid((e1 - e0 + 3) / 4);
#define GSIS_USWEEP(T, D, M) hipLaunchKernelGGL((k_usweep<T, D, M>), grid, dim3(256), 0, s, t.cases, nullptr, e0, e1)
#define GSIS_USWEEP_F(T, D) \
    do { \
        if (mf <= 4) GSIS_USWEEP(T, D, 4); \
        else if (mf <= 6) GSIS_USWEEP(T, D, 6); \
        else if (mf <= 8) GSIS_USWEEP(T, D, 8); \
        else GSIS_USWEEP(T, D, UMAXF); \
    } while (0)
        if (t.fp32) { if (t.dia) GSIS_USWEEP_F(float, true); else GSIS_USWEEP_F(float, false); }
        else { if (t.dia) GSIS_USWEEP_F(double, true); else GSIS_USWEEP_F(double, false); }
#undef GSIS_USWEEP_F
#undef GSIS_USWEEP
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

}  // namespace gsis

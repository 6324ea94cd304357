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
// density.  One wave per face, FP64 sums, lane partials combined by a fixed
// butterfly.
template <typename T>
__global__ __launch_bounds__(256) void k_uface_scale(GSIS_SPAN_ARGS)
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
        double out = 0.0, in = 0.0;
        for (int pos = lane; pos < g.nv; pos += 64) {
            const double *t = C.d.nt64 + 4 * (size_t)pos;
            const double xn = t[0] * nx + t[1] * ny + t[2] * nz;
            if (xn > 0.0) out += t[3] * xn * (double)f[pos];
            else if (xn < 0.0) in += t[3] * (-xn) * mb[pos];
        }
        scale = wave_sum(out) / wave_sum(in);
    }
    if (lane == 0) {
        C.d.ubf_s64[bf] = scale;
        C.d.ubf_s32[bf] = (float)scale;
    }
}

// Sweep entries [e0, e1) of one level: entry (cell << 8 | class), one wave each.
template <typename T, bool DIA>
__global__ __launch_bounds__(256) void k_usweep(GSIS_SPAN_ARGS, int e0, int e1)
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
    const int ent = ((cptr<int>)C.d.ulev)[e];
    const int cell = ent >> 8, cls = ent & 255;
    const cptr<int> cl = (cptr<int>)(C.d.ucls + cls);
    const unsigned mask = (unsigned)cl[0];
    const int pos0 = cl[1], cnt = cl[2];
    const cptr<T> par = (F32 ? (cptr<T>)C.d.parf : (cptr<T>)C.d.par) + (size_t)cell * NPAR;
    T p[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) p[k] = par[k];
    const cptr<int> coff = (cptr<int>)C.d.ucf_off;
    const int fb = coff[cell], nf = coff[cell + 1] - fb;
    const cptr<int> cnb = (cptr<int>)C.d.ucf_nb + fb;
    const cptr<int> cmeta = (cptr<int>)C.d.ucf_meta + fb;
    const cptr<T> ccoef = (F32 ? (cptr<T>)C.d.ucf_c32 : (cptr<T>)C.d.ucf_c64) + fb;
    const cptr<T> ori = F32 ? (cptr<T>)C.d.uori32 : (cptr<T>)C.d.uori64;
    const cptr<T> bsc = F32 ? (cptr<T>)C.d.ubf_s32 : (cptr<T>)C.d.ubf_s64;
    const gptr<const T> nt = F32 ? (gptr<const T>)C.d.nt32 : (gptr<const T>)C.d.nt64;
    const gptr<const T> mb = F32 ? (gptr<const T>)C.d.mb32 : (gptr<const T>)C.d.mb64;
    const gptr<const T> mb1 = F32 ? (gptr<const T>)C.d.mb1_32 : (gptr<const T>)C.d.mb1_64;
    const size_t nv = (size_t)g.nv;
    const gptr<T> f0 = (gptr<T>)C.d.f0, f1 = (gptr<T>)C.d.f1;
    const T idt = (T)g.inv_dt;
    const T invtau = DIA ? p[33] : p[13];

    // the faces of the cell: which bring the class's nodes in, and from where
    int src[UMAXF];      // cell row of an interior inflow face, or -1 - boundary face
    bool in[UMAXF];
    T on[UMAXF][3], cf[UMAXF];
#pragma unroll
    for (int j = 0; j < UMAXF; ++j) {
        if (j < nf) {
            const int meta = cmeta[j], k = meta & 31;
            const bool flip = (meta >> 5) & 1;
            in[j] = (((mask >> k) & 1u) != 0) == flip;   // xi . n out of the cell < 0 for the class
            src[j] = cnb[j];
            on[j][0] = ori[4 * k];
            on[j][1] = ori[4 * k + 1];
            on[j][2] = ori[4 * k + 2];
            cf[j] = ccoef[j];
        } else {
            in[j] = false;
            src[j] = 0;
            on[j][0] = on[j][1] = on[j][2] = cf[j] = T(0);
        }
    }
    for (int l0 = 0; l0 < cnt; l0 += 64) {
        const int l = l0 + lane;
        const bool active = l < cnt;
        const size_t pos = (size_t)pos0 + (active ? l : 0);
        const T xix = nt[4 * pos], xiy = nt[4 * pos + 1], xiz = nt[4 * pos + 2];
        // the inflow values first (independent loads), then the arithmetic
        T F0[UMAXF], F1[UMAXF];
#pragma unroll
        for (int j = 0; j < UMAXF; ++j) {
            F0[j] = F1[j] = T(0);
            if (j < nf && in[j]) {
                if (src[j] >= 0) {
                    F0[j] = f0[(size_t)src[j] * nv + pos];
                    if (DIA) F1[j] = f1[(size_t)src[j] * nv + pos];
                } else {
                    const int bfi = -1 - src[j];
                    const int slot = (cmeta[j] >> 6) & 7;
                    const T sc = bsc[bfi];
                    F0[j] = sc * mb[(size_t)slot * nv + pos];
                    if (DIA) F1[j] = sc * mb1[(size_t)slot * nv + pos];
                }
            }
        }
        T own0 = T(0), own1 = T(0);
        if (g.inv_dt != 0.0) {
            own0 = f0[(size_t)cell * nv + pos];
            if (DIA) own1 = f1[(size_t)cell * nv + pos];
        }
        const T cx = xix - p[0], cy = xiy - p[1], cz = xiz - p[2];
        T num0, num1 = T(0);
        if (DIA) ref_dia<T>(p, cx, cy, cz, p[3], p[4], num0, num1);
        else num0 = ref_mono<T>(p, cx, cy, cz, p[3]);
        num0 = fma(idt, own0, num0);
        if (DIA) num1 = fma(idt, own1, num1);
        T den = idt + invtau;
#pragma unroll
        for (int j = 0; j < UMAXF; ++j) {
            if (j < nf) {
                const T xn = fma(xiz, on[j][2], fma(xiy, on[j][1], xix * on[j][0]));
                const T a = fabs(xn) * cf[j];
                if (in[j]) {
                    num0 = fma(a, F0[j], num0);
                    if (DIA) num1 = fma(a, F1[j], num1);
                } else {
                    den += a;
                }
            }
        }
        if (active) {
            f0[(size_t)cell * nv + pos] = Arith<T>::div(num0, den);
            if (DIA) f1[(size_t)cell * nv + pos] = Arith<T>::div(num1, den);
        }
    }
}

hipError_t launch_uface_scale(const Target &t, hipStream_t s)
{
    const Geo &g = t.host->g;
    if (g.unbf == 0) return hipSuccess;
    const dim3 grid((g.unbf + 3) / 4);
    if (t.fp32) hipLaunchKernelGGL(k_uface_scale<float>, grid, dim3(256), 0, s, t.cases, nullptr);
    else hipLaunchKernelGGL(k_uface_scale<double>, grid, dim3(256), 0, s, t.cases, nullptr);
    return hipGetLastError();
}

hipError_t launch_usweep(const Target &t, const int *lev_off, int nlev, hipStream_t s)
{
    for (int L = 0; L < nlev; ++L) {
        const int e0 = lev_off[L], e1 = lev_off[L + 1];
        if (e1 <= e0) continue;
        const dim3 grid((e1 - e0 + 3) / 4);
#define GSIS_USWEEP(T, D) hipLaunchKernelGGL((k_usweep<T, D>), grid, dim3(256), 0, s, t.cases, nullptr, e0, e1)
        if (t.fp32) { if (t.dia) GSIS_USWEEP(float, true); else GSIS_USWEEP(float, false); }
        else { if (t.dia) GSIS_USWEEP(double, true); else GSIS_USWEEP(double, false); }
#undef GSIS_USWEEP
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

}  // namespace gsis

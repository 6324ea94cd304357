// GSIS-II macroscopic synthetic solve (Sec. 3.3), plain point-Jacobi
// iteration on the GPU.  Not an optimisation target: per-cell kernels.
//
// Unknowns per fluid cell W = (rho, rho u, E, Er) with E = rho |u|^2 + 1.5 rho Tt + Er,
// Er = (dr/2) rho Tr (monatomic: Er = 0) -- the moments 1, xi, |xi|^2 (+ 1 on
// f1) of the kinetic equation, so the face fluxes are mass rho u_n; momentum
// rho u u_n + (p n + sigma.n)/2; energy (E + p) u_n + (sigma.n).u + q.n + qr.n;
// Er u_n + qr.n, p = rho Tt.
// Stress and heat flux follow Eq. (full_constitutive): the NSF laws of
// Eq. (NSF_constitutive) at the iterate plus the high-order terms frozen at
// each face, HoT = (K_i + K_j)/2 - NSF_face(W^{n+1/2}).  In these units
// sigma_NSF = -(Tt^omega/delta)(grad u + grad u^T - (2/3) div u I),
// q_NSF = -(k_t Tt^omega/delta) grad Tt, qr_NSF = -(k_r Tt^omega/delta) grad Tr,
// [k_t; k_r] = A^{-1}[5; dr]/4 (Eq. mu_kappa), k_t = 15/8 for Pr = 2/3.
// Face gradients: normal difference, tangential = mean of the cells' central
// (one-sided at non-fluid neighbours) gradients.  Convective flux: Rusanov.
// Boundary faces: F_kin + F_eq(W^m) - F_eq(W^{n+1/2}) -- the kinetic flux of
// f^{n+1/2} keeps its non-equilibrium part while the equilibrium part
// follows the iterate -- or, with the Grad-13 wall flux, the same with the
// flux of the Grad-13 distributions of Eq. (G13_VDF) in place of F_eq, built
// from the iterate and the stress and heat fluxes of Eq. (full_constitutive)
// at the cell (NSF from its central gradients plus HoT_c, the kinetic values
// of f^{n+1/2} minus the NSF values at W^{n+1/2}).  Pseudo time: the diagonal of Eq. (res_macro),
// D_i = 1/dtau_i + (1/2) sum_faces Gamma / h, Gamma = s + C_d Tt^omega/(delta rho h),
// with one global step D* = max_i D_i per iteration so the update is exactly
// conservative, and the rotational relaxation 1/(Z tau) on the Er row.
#include "gsis_common.h"
#include "gsis_launch.h"

#include <algorithm>

namespace gsis {

// prims per cell: rho, ux, uy, uz, Tt, Tr, E, Er, c_s, Tt^omega / delta, 1/tau, (unused)
constexpr int NP = 12;

// The per-cell (per-face) arrays of the macroscopic solve are structures of
// arrays: field k of item i at buf[k * n + i], so the lanes of a wave, which
// take consecutive cells, read consecutive words.  Soa is one item's view.
// Every buffer is read and written through global-address-space pointers
// (gptr), so the loads and stores are global rather than flat instructions.
template <typename T> struct Soa {
    gptr<T> p;
    size_t n;
    __device__ __forceinline__ GSIS_GLOBAL_AS T &operator[](int k) const { return p[(size_t)k * n]; }
};
template <typename T> __device__ __forceinline__ Soa<T> soa(T *buf, size_t n, int i) { return Soa<T>{(gptr<T>)buf + i, n}; }
template <typename T> __device__ __forceinline__ Soa<T> soa(gptr<T> buf, size_t n, int i) { return Soa<T>{buf + i, n}; }
template <typename T> __device__ __forceinline__ gptr<T> G(T *p) { return (gptr<T>)p; }

template <class PV>
__device__ __forceinline__ void prim_from_W(const Geo &g, const double *W, PV P)
{
    double rho = W[0], irho = 1.0 / rho;
    double u0 = W[1] * irho, u1 = W[2] * irho, u2 = W[3] * irho;
    double E = W[4];
    double Er = g.species == 1 ? W[5] : 0.0;
    double uu = u0 * u0 + u1 * u1 + u2 * u2;
    double Tt = (2.0 / 3.0) * (E - Er - rho * uu) * irho;
    double Tr = g.species == 1 ? 2.0 * Er / (g.dr * rho) : Tt;
    P[0] = rho; P[1] = u0; P[2] = u1; P[3] = u2; P[4] = Tt; P[5] = Tr; P[6] = E; P[7] = Er;
    P[8] = sqrt(g.gam * Tt / 2.0);
    const double tw = pow_pos(Tt, g.omega);
    P[9] = tw / g.delta;
    P[10] = g.delta * rho * Tt / tw;
    P[11] = 0.0;
}

template <class PV, class GV>
__device__ __forceinline__ void nsf_face(const Geo &g, const PV &L, const PV &R, const GV &gL, const GV &gR, int a,
                                         double ih, double mu, double sigN[3], double *qN, double *qrN)
{
    double G[9];
    for (int b = 0; b < 3; ++b)
        for (int c = 0; c < 3; ++c)
            G[b * 3 + c] = (c == a) ? (R[1 + b] - L[1 + b]) * ih : 0.5 * (gL[b * 3 + c] + gR[b * 3 + c]);
    double div = G[0] + G[4] + G[8];
    for (int b = 0; b < 3; ++b)
        sigN[b] = -mu * (G[b * 3 + a] + G[a * 3 + b] - (b == a ? (2.0 / 3.0) * div : 0.0));
    *qN = -g.kt * mu * (R[4] - L[4]) * ih;
    *qrN = g.species == 1 ? -g.kr * mu * (R[5] - L[5]) * ih : 0.0;
}

// convective flux vector Phi(W).n and the state vector of one side
template <class PV>
__device__ __forceinline__ void side(const PV &P, int a, double Phi[6], double Wv[6])
{
    double rho = P[0], un = P[1 + a], p = P[0] * P[4];
    Phi[0] = rho * un;
#pragma unroll
    for (int b = 0; b < 3; ++b) Phi[1 + b] = rho * P[1 + b] * un + (b == a ? 0.5 * p : 0.0);
    Phi[4] = (P[6] + p) * un;
    Phi[5] = P[7] * un;
    Wv[0] = rho;
#pragma unroll
    for (int b = 0; b < 3; ++b) Wv[1 + b] = rho * P[1 + b];
    Wv[4] = P[6];
    Wv[5] = P[7];
}

// Macroscopic flux (Rusanov + NSF, no high-order terms) across the face from
// L to R = L + e_a.
template <class PV, class GV>
__device__ __forceinline__ void face_flux(const Geo &g, const PV &L, const PV &R, const GV &gL, const GV &gR, int a,
                                          double ih, bool euler, double F[6], double *Gam)
{
    const double TF = 0.5 * (L[4] + R[4]), rF = 0.5 * (L[0] + R[0]);
    // Euler constitutive relations: no stress or heat flux, no diffusive part in Gamma
    const double mu = euler ? 0.0 : pow_pos(TF, g.omega) / g.delta;
    double sigN[3] = {0.0, 0.0, 0.0}, qN = 0.0, qrN = 0.0;
    if (!euler) nsf_face(g, L, R, gL, gR, a, ih, mu, sigN, &qN, &qrN);
    double PhiL[6], WL[6], PhiR[6], WR[6];
    side(L, a, PhiL, WL);
    side(R, a, PhiR, WR);
    double sL = fabs(L[1 + a]) + L[8], sR = fabs(R[1 + a]) + R[8];
    double smax = sL > sR ? sL : sR;
#pragma unroll
    for (int k = 0; k < 6; ++k) F[k] = 0.5 * (PhiL[k] + PhiR[k]) - 0.5 * smax * (WR[k] - WL[k]);
    double uF[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) uF[b] = 0.5 * (L[1 + b] + R[1 + b]);
    const double qrn = g.species == 1 ? qrN : 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) F[1 + b] += 0.5 * sigN[b];
    F[4] += sigN[0] * uF[0] + sigN[1] * uF[1] + sigN[2] * uF[2] + qN + qrn;
    F[5] += qrn;
    *Gam = euler ? smax : smax + g.Cd * mu * ih / rF;
}

// Outgoing half-range psi-moments of M(rho, u, Tt) through face dir (sum over
// nodes with xi.n > 0 of w (xi.n) psi M), separable on the tensor grid and
// summed node by node on a node list, and
// the face flux of the equilibrium state with the face's boundary rule.  A
// group of FG adjacent lanes evaluates one face: the lanes share the nodes of
// each axis and a butterfly inside the group combines them, so every lane of
// the group ends with the result.
constexpr int FG = 8;

// gradient blocks of k_mac_grad and k_mac_advance: one (cell, axis) per
// thread, 256 threads, axis-major (a block holds one axis of 256 cells), so a
// wave's neighbour reads are coalesced and its work is uniform
__host__ __device__ inline int grad_axis_blocks(const Geo &g) { return (g.ncell + 255) / 256; }
__host__ __device__ inline int grad_blocks(const Geo &g) { return 3 * grad_axis_blocks(g); }
// boundary-face blocks (FG lanes per face); they come first in a launch that
// also has gradient blocks, so the longer face work starts first
__host__ __device__ inline int face_blocks(const Geo &g) { return (g.nface * FG + 255) / 256; }

__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int m = 1; m < FG; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

template <class PV>
__device__ void group_equilibrium_flux(const Geo &g, const BcInfo &bc, const Dev &d, const PV &P, int dir, int b,
                                       int sub, double F[6])
{
    const int a = dir / 2;
    const double sg = (dir & 1) ? 1.0 : -1.0;
    const double T = P[4], iT = 1.0 / T;
    const double piT = PI * T;
    const double K = P[0] / (piT * sqrt(piT)) * sg;
    const double h1 = g.species == 1 ? 0.5 * g.dr * P[5] : 0.0;
    const gptr<const double> in = G((const double *)d.inpsi) + (b * 6 + dir) * 6;
    double out[6];
    if (g.vlist) {
        // node list: the half-range sums over the outgoing nodes directly
        double s0 = 0.0, s1[3] = {0.0, 0.0, 0.0}, s4 = 0.0;
        const gptr<const double> nt = G((const double *)d.nt64);
        for (int k = sub; k < g.nv; k += FG) {
            const double x = nt[4 * (size_t)k + a];
            if (!(sg * x > 0.0)) continue;
            const double v0 = nt[4 * (size_t)k], v1 = nt[4 * (size_t)k + 1], v2 = nt[4 * (size_t)k + 2];
            const double cx = v0 - P[1], cy = v1 - P[2], cz = v2 - P[3];
            const double ex = nt[4 * (size_t)k + 3] * exp_core(fmax(-(cx * cx + cy * cy + cz * cz) * iT, -745.0)) * x;
            s0 += ex;
            s1[0] += ex * v0;
            s1[1] += ex * v1;
            s1[2] += ex * v2;
            s4 += ex * (v0 * v0 + v1 * v1 + v2 * v2);
        }
        s0 = group_sum(s0);
#pragma unroll
        for (int q = 0; q < 3; ++q) s1[q] = group_sum(s1[q]);
        s4 = group_sum(s4);
        out[0] = K * s0;
#pragma unroll
        for (int q = 0; q < 3; ++q) out[1 + q] = K * s1[q];
        out[4] = K * s4 + h1 * out[0];
        out[5] = h1 * out[0];
        const double sc = bc.kind[b] == 1 ? bc.rho[b] : out[0] / (-in[0]);
#pragma unroll
        for (int k = 0; k < 6; ++k) F[k] = out[k] + sc * in[k];
        return;
    }
    const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
    double H1 = 0, H2 = 0, H3 = 0;
    for (int k = sub; k < g.n1[a]; k += FG) {
        const double x = G(d.xi64[a])[k];
        if (!(sg * x > 0.0)) continue;
        const double c = x - P[1 + a];
        const double e = G(d.w64[a])[k] * exp_core(fmax(-c * c * iT, -745.0));
        H1 += e * x;
        H2 += e * x * x;
        H3 += e * x * x * x;
    }
    double S[2][3] = {{0, 0, 0}, {0, 0, 0}};
    const int ax2[2] = {b1, b2};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int ax = ax2[q];
        for (int k = sub; k < g.n1[ax]; k += FG) {
            const double x = G(d.xi64[ax])[k], c = x - P[1 + ax];
            const double e = G(d.w64[ax])[k] * exp_core(fmax(-c * c * iT, -745.0));
            S[q][0] += e;
            S[q][1] += e * x;
            S[q][2] += e * x * x;
        }
    }
    H1 = group_sum(H1);
    H2 = group_sum(H2);
    H3 = group_sum(H3);
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int p = 0; p < 3; ++p) S[q][p] = group_sum(S[q][p]);
    out[0] = K * H1 * S[0][0] * S[1][0];
    out[1 + a] = K * H2 * S[0][0] * S[1][0];
    out[1 + b1] = K * H1 * S[0][1] * S[1][0];
    out[1 + b2] = K * H1 * S[0][0] * S[1][1];
    out[4] = K * (H3 * S[0][0] * S[1][0] + H1 * S[0][2] * S[1][0] + H1 * S[0][0] * S[1][2]) + h1 * out[0];
    out[5] = h1 * out[0];
    const double sc = bc.kind[b] == 1 ? bc.rho[b] : out[0] / (-in[0]);
#pragma unroll
    for (int k = 0; k < 6; ++k) F[k] = out[k] + sc * in[k];
}

// Stress and heat fluxes of Eq. (NSF_constitutive) at the face group's cell
// from its central gradients (one-sided next to a non-fluid neighbour, zero
// with none): lane sub of the group holds v = (ux, uy, uz, Tt, Tr) of the
// cell's neighbour across direction sub (0..5; the cell's own state, with
// has = false, where that is not a fluid cell), lanes 6 and 7 the cell's own;
// mu = Tt^omega / delta of the cell.  sq = (sigma xx yy zz xy xz yz, q, qr),
// the same in every lane of the group.
__device__ __forceinline__ void group_cell_nsf(const Geo &g, const double v[5], bool has, double mu, double sq[12])
{
    const int base = (int)(threadIdx.x & 63) & ~(FG - 1);
    double Gu[9], gt[3], gr[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int hm = __shfl((int)has, base + 2 * a, 64), hp = __shfl((int)has, base + 2 * a + 1, 64);
        const double iden = (hm && hp) ? 0.5 * g.invh[a] : g.invh[a];
        const bool none = !hm && !hp;
        double dv[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) dv[k] = __shfl(v[k], base + 2 * a + 1, 64) - __shfl(v[k], base + 2 * a, 64);
#pragma unroll
        for (int b = 0; b < 3; ++b) Gu[b * 3 + a] = none ? 0.0 : dv[b] * iden;
        gt[a] = none ? 0.0 : dv[3] * iden;
        gr[a] = none ? 0.0 : dv[4] * iden;
    }
    const double div = Gu[0] + Gu[4] + Gu[8];
    sq[0] = -mu * (2.0 * Gu[0] - (2.0 / 3.0) * div);
    sq[1] = -mu * (2.0 * Gu[4] - (2.0 / 3.0) * div);
    sq[2] = -mu * (2.0 * Gu[8] - (2.0 / 3.0) * div);
    sq[3] = -mu * (Gu[1] + Gu[3]);
    sq[4] = -mu * (Gu[2] + Gu[6]);
    sq[5] = -mu * (Gu[5] + Gu[7]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        sq[6 + a] = -g.kt * mu * gt[a];
        sq[9 + a] = g.species == 1 ? -g.kr * mu * gr[a] : 0.0;
    }
}

// sum over the outgoing half of w xi_n c^e B(c) M(c) / (rho (pi T)^{-3/2}) on
// the tensor grid, c in the face's axes (normal, t1, t2), B the Grad-13
// bracket 1 + cs sigma:cc + cq (q.c)(c5 |c|^2 - 1): products of the 1-D sums
// N[i] = sum_{out} w e xi_n c_n^i and S1[j], S2[k] = sum w e c_t^j over the
// tangential axes (e the 1-D Gaussian factor).
template <int EN, int E1, int E2>
__device__ __forceinline__ double g13_bsum(const double N[6], const double S1[6], const double S2[6],
                                           const double sl[3][3], const double ql[3], double cs, double cq, double c5)
{
#define GSIS_A3(i, j, k) (N[(i) + EN] * S1[(j) + E1] * S2[(k) + E2])
    double r = GSIS_A3(0, 0, 0);
    r += cs * (sl[0][0] * GSIS_A3(2, 0, 0) + sl[1][1] * GSIS_A3(0, 2, 0) + sl[2][2] * GSIS_A3(0, 0, 2)
               + 2.0 * (sl[0][1] * GSIS_A3(1, 1, 0) + sl[0][2] * GSIS_A3(1, 0, 1) + sl[1][2] * GSIS_A3(0, 1, 1)));
    const double t = ql[0] * (c5 * (GSIS_A3(3, 0, 0) + GSIS_A3(1, 2, 0) + GSIS_A3(1, 0, 2)) - GSIS_A3(1, 0, 0))
                   + ql[1] * (c5 * (GSIS_A3(2, 1, 0) + GSIS_A3(0, 3, 0) + GSIS_A3(0, 1, 2)) - GSIS_A3(0, 1, 0))
                   + ql[2] * (c5 * (GSIS_A3(2, 0, 1) + GSIS_A3(0, 2, 1) + GSIS_A3(0, 0, 3)) - GSIS_A3(0, 0, 1));
#undef GSIS_A3
    return r + cq * t;
}

// The Grad-13 half-range sums of group_g13_flux on the tensor grid for a face
// normal to axis A (a compile-time constant, so that every stress and heat-flux
// component is picked by a constant index): out[6] before the boundary rule.
template <int A>
__device__ __forceinline__ void g13_tensor_flux(const Geo &g, const Dev &d, const double u[3], const double sq[12],
                                                double sg, double iT, double K, double cs, double cq, double c5,
                                                double cr, double h1, bool dia, int sub, double out[6])
{
    constexpr int T1 = (A + 1) % 3, T2 = (A + 2) % 3;
    constexpr int ax[3] = {A, T1, T2};
    // sq slot of sigma_{pq} in the face's axes: the diagonal 0..2, xy 3, xz 4, yz 5
    auto sslot = [](int x, int y) constexpr { return x == y ? x : 2 + x + y; };
    double N[6] = {0, 0, 0, 0, 0, 0}, S1[6] = {0, 0, 0, 0, 0, 0}, S2[6] = {0, 0, 0, 0, 0, 0};
    for (int k = sub; k < g.n1[A]; k += FG) {
        const double x = G(d.xi64[A])[k];
        if (!(sg * x > 0.0)) continue;
        const double c = x - u[A];
        double e = G(d.w64[A])[k] * exp_core(fmax(-c * c * iT, -745.0)) * x;
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            N[p] += e;
            e *= c;
        }
    }
    for (int k = sub; k < g.n1[T1]; k += FG) {
        const double c = G(d.xi64[T1])[k] - u[T1];
        double e = G(d.w64[T1])[k] * exp_core(fmax(-c * c * iT, -745.0));
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            S1[p] += e;
            e *= c;
        }
    }
    for (int k = sub; k < g.n1[T2]; k += FG) {
        const double c = G(d.xi64[T2])[k] - u[T2];
        double e = G(d.w64[T2])[k] * exp_core(fmax(-c * c * iT, -745.0));
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            S2[p] += e;
            e *= c;
        }
    }
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        N[p] = group_sum(N[p]);
        S1[p] = group_sum(S1[p]);
        S2[p] = group_sum(S2[p]);
    }
    double sl[3][3], ql[3], rl[3], ul[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
#pragma unroll
        for (int q = 0; q < 3; ++q) sl[p][q] = sq[sslot(ax[p], ax[q])];
        ql[p] = sq[6 + ax[p]];
        rl[p] = sq[9 + ax[p]];
        ul[p] = u[ax[p]];
    }
    const double b0 = g13_bsum<0, 0, 0>(N, S1, S2, sl, ql, cs, cq, c5);
    const double bn = g13_bsum<1, 0, 0>(N, S1, S2, sl, ql, cs, cq, c5);
    const double b1 = g13_bsum<0, 1, 0>(N, S1, S2, sl, ql, cs, cq, c5);
    const double b2 = g13_bsum<0, 0, 1>(N, S1, S2, sl, ql, cs, cq, c5);
    const double bnn = g13_bsum<2, 0, 0>(N, S1, S2, sl, ql, cs, cq, c5);
    const double b11 = g13_bsum<0, 2, 0>(N, S1, S2, sl, ql, cs, cq, c5);
    const double b22 = g13_bsum<0, 0, 2>(N, S1, S2, sl, ql, cs, cq, c5);
    out[0] = K * b0;
    out[1 + A] = K * (bn + ul[0] * b0);
    out[1 + T1] = K * (b1 + ul[1] * b0);
    out[1 + T2] = K * (b2 + ul[2] * b0);
    const double uu = ul[0] * ul[0] + ul[1] * ul[1] + ul[2] * ul[2];
    const double e0 = bnn + b11 + b22 + 2.0 * (ul[0] * bn + ul[1] * b1 + ul[2] * b2) + uu * b0;
    const double sr = rl[0] * N[1] * S1[0] * S2[0] + rl[1] * N[0] * S1[1] * S2[0] + rl[2] * N[0] * S1[0] * S2[1];
    const double f1 = dia ? K * (h1 * b0 + cr * sr) : 0.0;
    out[4] = K * e0 + f1;
    out[5] = f1;
}

// The flux of boundary face dir when the cell holds the Grad-13 distributions
// of Eq. (G13_VDF) of its state P and sq = (sigma, q, qr) (Eq. GSIS-DVM-flux),
// with the face's boundary rule (a wall's density from zero net mass flux):
//   f0 = M [1 + sigma:cc / (rho Tt^2) + 2 (q.c) / (rho Tt^2) (2 |c|^2 / (5 Tt) - 1)],
//   f1 = (dr/2) Tr f0 + 2 M (qr.c) / (rho Tt),
// velocities in sqrt(2 R T0) (these forms give back rho, u, Tt, sigma, q, Tr
// and qr as the moments of Eq. getmoment).  A group of FG lanes per face, as
// group_equilibrium_flux.
template <class PV>
__device__ __forceinline__ void group_g13_flux(const Geo &g, const BcInfo &bc, const Dev &d, const PV &P, const double sq[12], int dir,
                               int b, int sub, double F[6])
{
    const int a = dir / 2;
    const double sg = (dir & 1) ? 1.0 : -1.0;
    const double T = P[4], iT = 1.0 / T;
    const double piT = PI * T;
    const double K = P[0] / (piT * sqrt(piT)) * sg;
    const double u[3] = {P[1], P[2], P[3]};
    const double irT2 = 1.0 / (P[0] * T * T);
    const double cs = irT2, cq = 2.0 * irT2, c5 = 2.0 / (5.0 * T);
    const double cr = 2.0 / (P[0] * T);
    const bool dia = g.species == 1;
    const double h1 = dia ? 0.5 * g.dr * P[5] : 0.0;
    const gptr<const double> in = G((const double *)d.inpsi) + (b * 6 + dir) * 6;
    double out[6];
    if (g.vlist) {
        double s0 = 0.0, s1[3] = {0.0, 0.0, 0.0}, s4 = 0.0, sr = 0.0;
        const gptr<const double> nt = G((const double *)d.nt64);
        for (int k = sub; k < g.nv; k += FG) {
            const double x = nt[4 * (size_t)k + a];
            if (!(sg * x > 0.0)) continue;
            const double v0 = nt[4 * (size_t)k], v1 = nt[4 * (size_t)k + 1], v2 = nt[4 * (size_t)k + 2];
            const double cx = v0 - u[0], cy = v1 - u[1], cz = v2 - u[2];
            const double cc = cx * cx + cy * cy + cz * cz;
            const double e = nt[4 * (size_t)k + 3] * exp_core(fmax(-cc * iT, -745.0)) * x;
            const double scc = sq[0] * cx * cx + sq[1] * cy * cy + sq[2] * cz * cz
                             + 2.0 * (sq[3] * cx * cy + sq[4] * cx * cz + sq[5] * cy * cz);
            const double qc = sq[6] * cx + sq[7] * cy + sq[8] * cz;
            const double eb = e * (1.0 + cs * scc + cq * qc * (c5 * cc - 1.0));
            s0 += eb;
            s1[0] += eb * v0;
            s1[1] += eb * v1;
            s1[2] += eb * v2;
            s4 += eb * (v0 * v0 + v1 * v1 + v2 * v2);
            if (dia) sr += e * (sq[9] * cx + sq[10] * cy + sq[11] * cz);
        }
        s0 = group_sum(s0);
#pragma unroll
        for (int q = 0; q < 3; ++q) s1[q] = group_sum(s1[q]);
        s4 = group_sum(s4);
        sr = group_sum(sr);
        out[0] = K * s0;
#pragma unroll
        for (int q = 0; q < 3; ++q) out[1 + q] = K * s1[q];
        const double f1 = dia ? K * (h1 * s0 + cr * sr) : 0.0;
        out[4] = K * s4 + f1;
        out[5] = f1;
    } else {
        if (a == 0) g13_tensor_flux<0>(g, d, u, sq, sg, iT, K, cs, cq, c5, cr, h1, dia, sub, out);
        else if (a == 1) g13_tensor_flux<1>(g, d, u, sq, sg, iT, K, cs, cq, c5, cr, h1, dia, sub, out);
        else g13_tensor_flux<2>(g, d, u, sq, sg, iT, K, cs, cq, c5, cr, h1, dia, sub, out);
    }
    const double sc = bc.kind[b] == 1 ? bc.rho[b] : out[0] / (-in[0]);
#pragma unroll
    for (int k = 0; k < 6; ++k) F[k] = out[k] + sc * in[k];
}

// Gamma of a boundary face: outward speed plus the diffusive term of the cell
template <class PV>
__device__ __forceinline__ double boundary_gamma(const Geo &g, const PV &P, int a, bool euler)
{
    return fabs(P[1 + a]) + P[8] + (euler ? 0.0 : g.Cd * P[9] / (P[0] * g.h[a]));
}

// W^{n+1/2} and the old half of the correction record.
__global__ __launch_bounds__(128) void k_mac_init(GSIS_SPAN_ARGS)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    int cell = blk * blockDim.x + threadIdx.x;
    if (cell >= g.ncell || !G(d.cflag)[cell]) return;
    const gptr<const double> m = G((const double *)d.cm) + (size_t)cell * NMOM;
    double rho = m[0], Tt = m[4];
    double uu = m[1] * m[1] + m[2] * m[2] + m[3] * m[3];
    double Er = g.species == 1 ? 0.5 * g.dr * rho * m[14] : 0.0;
    const size_t n = g.ncell;
    double W[6];
    W[0] = rho;
    W[1] = rho * m[1]; W[2] = rho * m[2]; W[3] = rho * m[3];
    W[4] = rho * uu + 1.5 * rho * Tt + Er;
    W[5] = Er;
    const Soa<double> Wd = soa(d.W, n, cell);
    for (int k = 0; k < 6; ++k) Wd[k] = W[k];
    const gptr<double> c = G(d.corr) + (size_t)cell * NCORR;
    c[6] = rho; c[7] = m[1]; c[8] = m[2]; c[9] = m[3]; c[10] = Tt;
    c[11] = g.species == 1 ? m[14] : Tt;
    prim_from_W(g, W, soa(d.P, n, cell));
}

// Column a of the velocity gradient of one cell: central differences, one-sided
// next to a non-fluid neighbour, zero with none.
__device__ void cell_grad_col(const Geo &g, const Dev &d, int cell, int a)
{
    const int nm = G(d.nbr)[(size_t)(2 * a) * g.ncell + cell], np = G(d.nbr)[(size_t)(2 * a + 1) * g.ncell + cell];
    const size_t n = g.ncell;
    const Soa<double> Pm = soa(d.P, n, nm >= 0 ? nm : cell);
    const Soa<double> Pp = soa(d.P, n, np >= 0 ? np : cell);
    const double iden = (nm >= 0 && np >= 0) ? 0.5 * g.invh[a] : g.invh[a];
    const Soa<double> G = soa(d.grad, n, cell);
#pragma unroll
    for (int b = 0; b < 3; ++b) G[b * 3 + a] = (nm < 0 && np < 0) ? 0.0 : (Pp[1 + b] - Pm[1 + b]) * iden;
}

// Blocks [0, nfb): boundary faces, FG lanes per face: F_b = fixed part +
// F_eq(W^m) and its Gamma (skipped when with_faces is 0).  Blocks [nfb, ...):
// central gradients of u, one (cell, axis) per thread.
__global__ __launch_bounds__(256) void k_mac_grad(GSIS_SPAN_ARGS, int with_faces, int euler)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    const BcInfo &bc = C.bc;
    const int nfb = face_blocks(g);
    if (blk >= nfb) {
        const int gb = blk - nfb, npa = grad_axis_blocks(g), a = gb / npa;
        const int cell = (gb - a * npa) * (int)blockDim.x + (int)threadIdx.x;
        if (cell < g.ncell && G(d.cflag)[cell]) cell_grad_col(g, d, cell, a);
        return;
    }
    if (!with_faces) return;
    // whole groups of FG lanes share f, so the group butterflies stay inside live lanes
    const int f = (blk * (int)blockDim.x + (int)threadIdx.x) / FG;
    const int sub = threadIdx.x & (FG - 1);
    if (f >= g.nface) return;
    const int cell = G(d.face_cell)[f], dir = G(d.face_dir)[f];
    const Soa<double> P = soa(d.P, g.ncell, cell);
    double Fe[6];
    group_equilibrium_flux(g, bc, d, P, dir, G(d.face_bc)[f], sub, Fe);
    if (sub < 6) G(d.Fb)[(size_t)sub * g.nface + f] = G(d.fbfix)[(size_t)sub * g.nface + f] + Fe[sub];
    if (sub == 7) G(d.Gb)[f] = boundary_gamma(g, P, dir / 2, euler);
}

// High-order terms at the faces (cell, cell + e_a), frozen at the kinetic
// state: the kinetic scheme's face flux of the moments of f^{n+1/2} (first-order
// upwind: the xi_a > 0 octant sums of the cell plus the xi_a < 0 octant sums of
// the neighbour) minus the macroscopic face flux at W^{n+1/2}, six values per
// face; the face flux of an iterate is its macroscopic flux plus these.  Zero
// for the Euler relations.
__global__ __launch_bounds__(128) void k_mac_hot(GSIS_SPAN_ARGS, int euler)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    int cell = blk * blockDim.x + threadIdx.x;
    if (cell >= g.ncell || !G(d.cflag)[cell]) return;
    const size_t n = g.ncell;
    const int m2row[3][3] = {{4, 7, 8}, {7, 5, 9}, {8, 9, 6}};
    for (int a = 0; a < 3; ++a) {
        const Soa<double> fx = soa(d.hot + (size_t)a * 6 * n, n, cell);
        const int nb = G(d.nbr)[(size_t)(2 * a + 1) * g.ncell + cell];
        if (euler || nb < 0) {
            for (int k = 0; k < 6; ++k) fx[k] = 0.0;
            continue;
        }
        double Fk[6] = {0, 0, 0, 0, 0, 0};
        for (int o = 0; o < 8; ++o) {
            const int up = ((o >> a) & 1) ? nb : cell;   // xi_a < 0: the neighbour's value enters the face
            const gptr<const double> m = G((const double *)d.mom8) + ((size_t)up * 8 + o) * NRS;
            Fk[0] += m[1 + a];
            for (int b = 0; b < 3; ++b) Fk[1 + b] += m[m2row[a][b]];
            Fk[4] += m[10 + a] + m[14 + a];
            Fk[5] += m[14 + a];
        }
        const Soa<double> PL = soa(d.P, n, cell), PR = soa(d.P, n, nb);
        double F[6], Gam;
        face_flux(g, PL, PR, soa(d.grad, n, cell), soa(d.grad, n, nb), a, g.invh[a], false, F, &Gam);
        for (int k = 0; k < 6; ++k) fx[k] = Fk[k] - F[k];
        if (g.species != 1) fx[5] = 0.0;
    }
}

// Fixed part of each boundary face flux, F_kin(f^{n+1/2}) - F_eq(W^{n+1/2}), and
// the face flux of the first inner iteration, fixed part + F_eq(W^{n+1/2}).
// One group of FG lanes per face.
// G13: compiled with the Grad-13 wall flux for the cases that take it (the
// plain instantiation keeps its registers for the common path).
template <bool G13>
__global__ __launch_bounds__(256) void k_mac_fbfix(GSIS_SPAN_ARGS, int euler)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    const BcInfo &bc = C.bc;
    const int f = (int)(blk * blockDim.x + threadIdx.x) / FG;
    const int sub = threadIdx.x & (FG - 1);
    if (f >= g.nface) return;
    const int cell = G(d.face_cell)[f], dir = G(d.face_dir)[f], b = G(d.face_bc)[f];
    const int a = dir / 2;
    const int neg = (dir & 1) ? 0 : 1;
    const double sg = neg ? -1.0 : 1.0;
    double out[6] = {0, 0, 0, 0, 0, 0};
    const int m2row[3][3] = {{4, 7, 8}, {7, 5, 9}, {8, 9, 6}};
    for (int o = 0; o < 8; ++o) {
        if (((o >> a) & 1) != neg) continue;
        const gptr<const double> m = G((const double *)d.mom8) + ((size_t)cell * 8 + o) * NRS;
        out[0] += m[1 + a];
        for (int c = 0; c < 3; ++c) out[1 + c] += m[m2row[a][c]];
        out[4] += m[10 + a] + m[14 + a];
        out[5] += m[14 + a];
    }
    for (int k = 0; k < 6; ++k) out[k] *= sg;
    const gptr<const double> in = G((const double *)d.inpsi) + (b * 6 + dir) * 6;
    const double sc = bc.kind[b] == 1 ? bc.rho[b] : out[0] / (-in[0]);
    const Soa<double> P = soa(d.P, g.ncell, cell);
    double Fe[6];
    if (G13 && g.wall_flux == 1 && !euler) {
        // Grad-13 wall flux: the cell's high-order terms, HoT_c = kinetic stress
        // and heat fluxes of f^{n+1/2} - NSF_c(W^{n+1/2}), kept per face, and the
        // flux of the distributions of NSF_c + HoT_c
        int who = cell;
        bool has = false;
        if (sub < 6) {
            const int nb = G(d.nbr)[(size_t)sub * g.ncell + cell];
            if (nb >= 0) { who = nb; has = true; }
        }
        const Soa<double> Pw = soa(d.P, g.ncell, who);
        const double v[5] = {Pw[1], Pw[2], Pw[3], Pw[4], Pw[5]};
        double sq[12];
        group_cell_nsf(g, v, has, P[9], sq);
        const gptr<const double> m = G((const double *)d.cm) + (size_t)cell * NMOM;
        const bool dia = g.species == 1;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            // cm: sigma at 5..10, q at 11..13, qr at 15..17
            const double kin = k < 9 ? m[5 + k] : (dia ? m[6 + k] : 0.0);
            const double hot = kin - sq[k];
            if ((k & (FG - 1)) == sub) G(d.ghot)[(size_t)k * g.nface + f] = hot;
            sq[k] += hot;
        }
        group_g13_flux(g, bc, d, P, sq, dir, b, sub, Fe);
    } else {
        group_equilibrium_flux(g, bc, d, P, dir, b, sub, Fe);
    }
    if (sub < 6) {
        // Euler: the boundary flux is the iterate's own F_eq, no fixed kinetic part
        const double fix = euler ? 0.0 : out[sub] + sc * in[sub] - Fe[sub];
        G(d.fbfix)[(size_t)sub * g.nface + f] = fix;
        G(d.Fb)[(size_t)sub * g.nface + f] = fix + Fe[sub];
    }
    if (sub == 7) G(d.Gb)[f] = boundary_gamma(g, P, a, euler);
}

// Flux of face dir of a cell divided by h (outward positive), and Gamma / h.
// dir is a compile-time constant so every index is static.
// Index of the neighbour across face dir on the uniform grid (cell -+ 1, nx,
// nx ny), clamped into the array: equal to the neighbour whenever the face is
// interior, and a valid address otherwise, so the neighbour's data can be
// loaded without waiting for the neighbour table.
__device__ __forceinline__ int grid_neighbour(const Geo &g, int cell, int dir)
{
    const int a = dir / 2;
    const int step = a == 0 ? 1 : (a == 1 ? g.nx : g.nx * g.ny);
    return (dir & 1) ? min(cell + step, g.ncell - 1) : max(cell - step, 0);
}

// With KEEP the cell's own prims 0..10 are also returned in own[], loaded with
// the face data, so the caller needs no second round trip to memory.
template <int DIR, int NW, bool KEEP, bool EULER>
__device__ __forceinline__ void face_term(const Geo &g, const Dev &d, int cell, double out[NW], double &gam,
                                          double *own)
{
    constexpr int a = DIR / 2;
    const double ih = g.invh[a];
    const size_t nc = g.ncell;
    // both sides' data into registers first, in parallel with the table lookup
    const int nb = grid_neighbour(g, cell, DIR);
    const int L = (DIR & 1) ? cell : nb, R = (DIR & 1) ? nb : cell;
    // only what the face flux reads: no Tr, Er, qr for the monatomic gas and no
    // normal gradient column (the normal derivative is the two-cell difference)
    constexpr bool DIA = NW == 6;
    double PL[NP], PR[NP], GL[9], GR[9], HO[6];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const bool use = DIA || (k != 5 && k != 7);
        PL[k] = use ? G(d.P)[(size_t)k * nc + L] : 0.0;
        PR[k] = use ? G(d.P)[(size_t)k * nc + R] : 0.0;
        const bool tan = k % 3 != a;
        GL[k] = tan ? G(d.grad)[(size_t)k * nc + L] : 0.0;
        GR[k] = tan ? G(d.grad)[(size_t)k * nc + R] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) HO[k] = (DIA || k < 5) ? G(d.hot)[(size_t)(a * 6 + k) * nc + L] : 0.0;
    if (KEEP) {
#pragma unroll
        for (int k = 0; k < 9; ++k) own[k] = (DIR & 1) ? PL[k] : PR[k];
        own[9] = G(d.P)[(size_t)9 * nc + cell];
        own[10] = G(d.P)[(size_t)10 * nc + cell];
    }
    const int n = G(d.nbr)[(size_t)DIR * g.ncell + cell];
    if (n >= 0) {
        double F[6], Gam;
        face_flux(g, PL, PR, GL, GR, a, ih, EULER, F, &Gam);
#pragma unroll
        for (int k = 0; k < NW; ++k) out[k] = ((DIR & 1) ? F[k] + HO[k] : -(F[k] + HO[k])) * ih;
        gam = Gam * ih;
    } else {
        const int f = -n - 1;
#pragma unroll
        for (int k = 0; k < NW; ++k) out[k] = G(d.Fb)[(size_t)k * g.nface + f] * ih;
        gam = G(d.Gb)[f] * ih;
    }
}

// Residual and diagonal of every cell; D* = max D_i by an atomic max on the
// bit pattern (positive doubles order like their bits), so it is exact and
// order independent.  A block holds 64 cells and six waves; wave j evaluates
// face j of every cell, LDS collects the six terms, and the first wave adds
// them in face order, finishes the cells and issues one atomic for the wave's
// largest D_i.
constexpr int RES_CELLS = 64;

// Six waves per SIMD (at most 80 VGPRs): four blocks per CU instead of three.
template <bool DIA, bool EULER>
__global__ __launch_bounds__(384) __attribute__((amdgpu_waves_per_eu(6))) void k_mac_res(GSIS_SPAN_ARGS, int slot)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;

    constexpr int NW = DIA ? 6 : 5;
    __shared__ double red[6][NW + 1][RES_CELLS];
    const int lane = threadIdx.x & 63;
    const int dir = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int cell = blk * RES_CELLS + lane;
    const bool live = cell < g.ncell && G(d.cflag)[cell];
    double out[NW], gam = 0.0, Pi[11];
#pragma unroll
    for (int k = 0; k < NW; ++k) out[k] = 0.0;
    if (live) {
        switch (dir) {
        case 0: face_term<0, NW, true, EULER>(g, d, cell, out, gam, Pi); break;
        case 1: face_term<1, NW, false, EULER>(g, d, cell, out, gam, nullptr); break;
        case 2: face_term<2, NW, false, EULER>(g, d, cell, out, gam, nullptr); break;
        case 3: face_term<3, NW, false, EULER>(g, d, cell, out, gam, nullptr); break;
        case 4: face_term<4, NW, false, EULER>(g, d, cell, out, gam, nullptr); break;
        default: face_term<5, NW, false, EULER>(g, d, cell, out, gam, nullptr); break;
        }
    }
#pragma unroll
    for (int k = 0; k < NW; ++k) red[dir][k][lane] = out[k];
    red[dir][NW][lane] = gam;
    __syncthreads();
    if (dir != 0) return;
    double D = 0.0;
    if (live) {
        double res[6], sumG = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) res[k] = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
#pragma unroll
            for (int k = 0; k < NW; ++k) res[k] -= red[j][k][lane];
            sumG += red[j][NW][lane];
        }
        const double invtau = Pi[10];
        if (DIA) {
            double T = (3.0 * Pi[4] + g.dr * Pi[5]) / (3.0 + g.dr);
            res[5] += 0.5 * g.dr * Pi[0] * (T - Pi[5]) * invtau / g.Zr;
        }
        double umag = sqrt(Pi[1] * Pi[1] + Pi[2] * Pi[2] + Pi[3] * Pi[3]);
        double idt = (umag + Pi[8] + (EULER ? 0.0 : g.Cd * Pi[9] / (Pi[0] * g.hmin))) / (g.macro_cfl * g.hmin);
        D = idt + 0.5 * sumG;
        const Soa<double> r = soa(d.R, g.ncell, cell);
#pragma unroll
        for (int k = 0; k < 6; ++k) r[k] = res[k];
        G(d.Src)[cell] = DIA ? invtau / g.Zr : 0.0;
        if (!(D > 0.0 && isfinite(D))) {
            atomicOr(d.errflag, 2);
            D = 0.0;
        }
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) D = fmax(D, __shfl_xor(D, m, 64));
    if (lane == 0 && D > 0.0)
        atomicMax(&d.dmax[(size_t)(slot * DSLOT + (blk & (DSLOT - 1))) * DSTRIDE],
                  (unsigned long long)__double_as_longlong(D));
}

// W of a cell after the pseudo-time step: W + R / D* (as R times 1/D*), the
// rotational-energy row with its relaxation source on the diagonal.
__device__ __forceinline__ void stepped_W(const Geo &g, const Dev &d, gptr<const double> Ws, int cell, double Dm, double iDm,
                                          double Wn[6])
{
    const Soa<const double> W = soa(Ws, g.ncell, cell);
    const Soa<double> r = soa(d.R, g.ncell, cell);
#pragma unroll
    for (int k = 0; k < 5; ++k) Wn[k] = W[k] + r[k] * iDm;
    Wn[5] = g.species == 1 ? W[5] + r[5] / (Dm + G(d.Src)[cell]) : W[5];
}

// Density and momentum rows of stepped_W only (what a neighbour's velocity needs).
__device__ __forceinline__ void stepped_mass_momentum(const Geo &g, const Dev &d, gptr<const double> Ws, int cell,
                                                      double iDm, double Wn[4])
{
    const Soa<const double> W = soa(Ws, g.ncell, cell);
    const Soa<double> r = soa(d.R, g.ncell, cell);
#pragma unroll
    for (int k = 0; k < 4; ++k) Wn[k] = W[k] + r[k] * iDm;
}

// End of an inner iteration: W' = W + R / D* with the new prims, and -- unless
// it is the last iteration -- the velocity gradient and the boundary-face
// fluxes of the new state, in one launch.  Grid as k_mac_grad: FG lanes per
// boundary face, then (cell, axis) threads (the axis-0 blocks also write W'
// and the prims).  Neighbours' new velocities and the face cells' new prims are
// formed from W and R directly, so W is double buffered (read src, write dst).
template <bool G13>
__global__ __launch_bounds__(256) void k_mac_advance(GSIS_SPAN_ARGS, int slot, int parity, int last, int euler)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    const BcInfo &bc = C.bc;
    const gptr<const double> Ws = G((const double *)(parity ? d.W2 : d.W));
    const gptr<double> Wd = G(parity ? d.W : d.W2);
    // D*: each lane loads one partial slot, the wave takes their max
    double Dm = __longlong_as_double((long long)G(d.dmax)[(size_t)(slot * DSLOT + (threadIdx.x & (DSLOT - 1))) * DSTRIDE]);
#pragma unroll
    for (int m = 1; m < DSLOT; m <<= 1) Dm = fmax(Dm, __shfl_xor(Dm, m, 64));
    const double iDm = 1.0 / Dm;
    const int nfb = face_blocks(g);
    if (blk >= nfb) {
        const int gb = blk - nfb;
        // the other slot was last used by the previous iteration
        if (gb == 0 && (int)threadIdx.x < DSLOT) G(d.dmax)[(size_t)((slot ^ 1) * DSLOT + threadIdx.x) * DSTRIDE] = 0ull;
        const int npa = grad_axis_blocks(g), a = gb / npa;
        if (a != 0 && last) return;
        const int cell = (gb - a * npa) * (int)blockDim.x + (int)threadIdx.x;
        if (cell >= g.ncell || !G(d.cflag)[cell]) return;
        double Wn[6];
        stepped_W(g, d, Ws, cell, Dm, iDm, Wn);
        if (a == 0) {
            const Soa<double> Wc = soa(Wd, g.ncell, cell);
#pragma unroll
            for (int k = 0; k < 6; ++k) Wc[k] = Wn[k];
            prim_from_W(g, Wn, soa(d.P, g.ncell, cell));
        }
        if (last) return;
        // neighbours' states loaded at grid indices, in parallel with the table lookup
        double Wm[4], Wp[4];
        stepped_mass_momentum(g, d, Ws, grid_neighbour(g, cell, 2 * a), iDm, Wm);
        stepped_mass_momentum(g, d, Ws, grid_neighbour(g, cell, 2 * a + 1), iDm, Wp);
        const int nm = G(d.nbr)[(size_t)(2 * a) * g.ncell + cell], np = G(d.nbr)[(size_t)(2 * a + 1) * g.ncell + cell];
        double um[3], up[3];
        const double ic = 1.0 / Wn[0], im = 1.0 / Wm[0], ip = 1.0 / Wp[0];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double uc = Wn[1 + b] * ic;
            um[b] = nm >= 0 ? Wm[1 + b] * im : uc;
            up[b] = np >= 0 ? Wp[1 + b] * ip : uc;
        }
        const double iden = (nm >= 0 && np >= 0) ? 0.5 * g.invh[a] : g.invh[a];
        const Soa<double> G = soa(d.grad, g.ncell, cell);
#pragma unroll
        for (int b = 0; b < 3; ++b) G[b * 3 + a] = (nm < 0 && np < 0) ? 0.0 : (up[b] - um[b]) * iden;
        return;
    }
    if (last) return;
    const int f = (blk * (int)blockDim.x + (int)threadIdx.x) / FG;
    const int sub = threadIdx.x & (FG - 1);
    if (f >= g.nface) return;
    const int cell = G(d.face_cell)[f], dir = G(d.face_dir)[f];
    double Wn[6], P[NP];
    stepped_W(g, d, Ws, cell, Dm, iDm, Wn);
    prim_from_W(g, Wn, P);
    double Fe[6];
    if (G13 && g.wall_flux == 1 && !euler) {
        // Grad-13 wall flux of the new state: NSF_c from the new states of the
        // cell and its neighbours (one per lane) plus the cell's HoT_c
        int who = cell;
        bool has = false;
        if (sub < 6) {
            const int nb = G(d.nbr)[(size_t)sub * g.ncell + cell];
            if (nb >= 0) { who = nb; has = true; }
        }
        double Ww[6];
        stepped_W(g, d, Ws, who, Dm, iDm, Ww);
        // u, Tt, Tr of the new state, as prim_from_W forms them
        const double irho = 1.0 / Ww[0];
        const double w0 = Ww[1] * irho, w1 = Ww[2] * irho, w2 = Ww[3] * irho;
        const double wEr = g.species == 1 ? Ww[5] : 0.0;
        const double wTt = (2.0 / 3.0) * (Ww[4] - wEr - Ww[0] * (w0 * w0 + w1 * w1 + w2 * w2)) * irho;
        const double v[5] = {w0, w1, w2, wTt, g.species == 1 ? 2.0 * wEr / (g.dr * Ww[0]) : wTt};
        double sq[12];
        group_cell_nsf(g, v, has, P[9], sq);
#pragma unroll
        for (int k = 0; k < 12; ++k) sq[k] += G(d.ghot)[(size_t)k * g.nface + f];
        group_g13_flux(g, bc, d, P, sq, dir, G(d.face_bc)[f], sub, Fe);
    } else {
        group_equilibrium_flux(g, bc, d, P, dir, G(d.face_bc)[f], sub, Fe);
    }
    if (sub < 6) G(d.Fb)[(size_t)sub * g.nface + f] = G(d.fbfix)[(size_t)sub * g.nface + f] + Fe[sub];
    if (sub == 7) G(d.Gb)[f] = boundary_gamma(g, P, dir / 2, euler);
}

// one block per case
__global__ void k_mac_reset(GSIS_SPAN_ARGS)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    for (int j = threadIdx.x; j < 2 * DSLOT; j += blockDim.x) G(C.d.dmax)[(size_t)j * DSTRIDE] = 0ull;
}

// New half of the correction record; flags non-physical states.
__global__ __launch_bounds__(128) void k_mac_final(GSIS_SPAN_ARGS)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    int cell = blk * blockDim.x + threadIdx.x;
    if (cell >= g.ncell || !G(d.cflag)[cell]) return;
    const Soa<double> P = soa(d.P, g.ncell, cell);
    const gptr<double> c = G(d.corr) + (size_t)cell * NCORR;
    c[0] = P[0]; c[1] = P[1]; c[2] = P[2]; c[3] = P[3]; c[4] = P[4];
    c[5] = g.species == 1 ? P[5] : P[4];
    if (!(P[0] > 0.0) || !(P[4] > 0.0) || !isfinite(P[6]) || (g.species == 1 && !(P[5] > 0.0))) atomicOr(d.errflag, 4);
}

hipError_t launch_gsis_macro(const Target &t, int iters, hipStream_t s, int euler)
{
    hipLaunchKernelGGL(k_mac_reset, dim3(t.nblk[K_CASE]), dim3(64), 0, s, GSIS_SPAN(t.span(K_CASE)));
    hipLaunchKernelGGL(k_mac_init, dim3(t.nblk[K_CELL128]), dim3(128), 0, s, GSIS_SPAN(t.span(K_CELL128)));
    hipLaunchKernelGGL(k_mac_grad, dim3(t.nblk[K_GRAD]), dim3(256), 0, s, GSIS_SPAN(t.span(K_GRAD)), 0, euler);
    hipLaunchKernelGGL(k_mac_hot, dim3(t.nblk[K_CELL128]), dim3(128), 0, s, GSIS_SPAN(t.span(K_CELL128)), euler);
    if (t.nblk[K_FACE8] > 0) {
        if (t.g13) hipLaunchKernelGGL(k_mac_fbfix<true>, dim3(t.nblk[K_FACE8]), dim3(256), 0, s, GSIS_SPAN(t.span(K_FACE8)), euler);
        else hipLaunchKernelGGL(k_mac_fbfix<false>, dim3(t.nblk[K_FACE8]), dim3(256), 0, s, GSIS_SPAN(t.span(K_FACE8)), euler);
    }
    for (int it = 0; it < iters; ++it) {
        const int slot = it & 1;
        // the Euler form is its own instantiation: a run-time flag costs the
        // residual registers (and spills) on the common path
        const dim3 gr(t.nblk[K_RES]), bl(384);
        const Span sp = t.span(K_RES);
        if (t.dia) {
            if (euler) hipLaunchKernelGGL((k_mac_res<true, true>), gr, bl, 0, s, GSIS_SPAN(sp), slot);
            else hipLaunchKernelGGL((k_mac_res<true, false>), gr, bl, 0, s, GSIS_SPAN(sp), slot);
        } else {
            if (euler) hipLaunchKernelGGL((k_mac_res<false, true>), gr, bl, 0, s, GSIS_SPAN(sp), slot);
            else hipLaunchKernelGGL((k_mac_res<false, false>), gr, bl, 0, s, GSIS_SPAN(sp), slot);
        }
        if (t.g13)
            hipLaunchKernelGGL(k_mac_advance<true>, dim3(t.nblk[K_GRAD]), dim3(256), 0, s, GSIS_SPAN(t.span(K_GRAD)), slot,
                               it & 1, it == iters - 1 ? 1 : 0, euler);
        else
            hipLaunchKernelGGL(k_mac_advance<false>, dim3(t.nblk[K_GRAD]), dim3(256), 0, s, GSIS_SPAN(t.span(K_GRAD)), slot,
                               it & 1, it == iters - 1 ? 1 : 0, euler);
    }
    hipLaunchKernelGGL(k_mac_final, dim3(t.nblk[K_CELL128]), dim3(128), 0, s, GSIS_SPAN(t.span(K_CELL128)));
    return hipGetLastError();
}

// ------------------------------------------------ unstructured mesh solve
// The same solve on an unstructured mesh (one case): faces of any normal n
// (out of the owner), area S, cells of volume V.  Velocity gradient of a cell
// by least squares over its face neighbours (weights from the host: the
// inverse of sum_j d_j d_j^T on its range applied to d_j), face gradient the
// mean of the two cells' corrected along d = x_R - x_L to the two-cell
// difference, normal heat fluxes -k mu (T_R - T_L) / h with h = d . n (twice
// the centroid-to-face distance along n on a boundary), Rusanov; fluxes per
// unit area times S / V in the residual and the diagonal; the high-order
// terms at every face the kinetic flux of f^{n+1/2} minus the macroscopic
// flux of W^{n+1/2}; on a boundary face F_kin + F_eq(W^m) - F_eq(W^{n+1/2}).

// Rusanov + NSF flux across face f from L to R (no high-order terms).
template <class PV, class GV>
__device__ __forceinline__ void uface_flux(const Geo &g, const PV &L, const PV &R, const GV &gL, const GV &gR,
                                           const double fg[9], bool euler, double F[6], double *Gam)
{
    const double n[3] = {fg[1], fg[2], fg[3]}, h = fg[4], dl = fg[5], e[3] = {fg[6], fg[7], fg[8]};
    const double TF = 0.5 * (L[4] + R[4]), rF = 0.5 * (L[0] + R[0]);
    // Euler constitutive relations: no stress or heat flux, no diffusive part in Gamma
    const double mu = euler ? 0.0 : pow_pos(TF, g.omega) / g.delta;
    double G[9];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        double gm[3], gd = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            gm[c] = 0.5 * (gL[b * 3 + c] + gR[b * 3 + c]);
            gd += gm[c] * e[c];
        }
        const double corr = (R[1 + b] - L[1 + b]) / dl - gd;
#pragma unroll
        for (int c = 0; c < 3; ++c) G[b * 3 + c] = gm[c] + corr * e[c];
    }
    const double div = G[0] + G[4] + G[8];
    double sN[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) acc += (G[b * 3 + c] + G[c * 3 + b]) * n[c];
        sN[b] = -mu * (acc - (2.0 / 3.0) * div * n[b]);
    }
    const double qN = -g.kt * mu * (R[4] - L[4]) / h;
    const double qrN = g.species == 1 ? -g.kr * mu * (R[5] - L[5]) / h : 0.0;
    double Phi[2][6], Wv[2][6], un[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const PV &P = k ? R : L;
        const double rho = P[0], p = P[0] * P[4];
        un[k] = P[1] * n[0] + P[2] * n[1] + P[3] * n[2];
        Phi[k][0] = rho * un[k];
#pragma unroll
        for (int b = 0; b < 3; ++b) Phi[k][1 + b] = rho * P[1 + b] * un[k] + 0.5 * p * n[b];
        Phi[k][4] = (P[6] + p) * un[k];
        Phi[k][5] = P[7] * un[k];
        Wv[k][0] = rho;
#pragma unroll
        for (int b = 0; b < 3; ++b) Wv[k][1 + b] = rho * P[1 + b];
        Wv[k][4] = P[6];
        Wv[k][5] = P[7];
    }
    const double sL = fabs(un[0]) + L[8], sR = fabs(un[1]) + R[8];
    const double smax = sL > sR ? sL : sR;
#pragma unroll
    for (int k = 0; k < 6; ++k) F[k] = 0.5 * (Phi[0][k] + Phi[1][k]) - 0.5 * smax * (Wv[1][k] - Wv[0][k]);
#pragma unroll
    for (int b = 0; b < 3; ++b) F[1 + b] += 0.5 * sN[b];
    F[4] += sN[0] * 0.5 * (L[1] + R[1]) + sN[1] * 0.5 * (L[2] + R[2]) + sN[2] * 0.5 * (L[3] + R[3]) + qN + qrN;
    F[5] += qrN;
    *Gam = euler ? smax : smax + g.Cd * mu / (rF * h);
}

// Velocity gradient of every cell: G[b][c] = sum over its interior face
// entries of (u_j - u_i)_b w_c.
__global__ __launch_bounds__(256) void k_umac_grad(GSIS_SPAN_ARGS)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    const int cell = blk * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    const size_t n = g.ncell;
    const Soa<double> P = soa(d.P, n, cell);
    const double ui[3] = {P[1], P[2], P[3]};
    double Gc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int first = G(d.ucf_first)[cell], cnt = G(d.ucf_first)[cell + 1] - first;
    for (int k = 0; k < cnt; ++k) {
        const int e = first + k;
        const int j = G(d.ucf_nb)[e];
        if (j < 0) continue;
        const Soa<double> Pj = soa(d.P, n, j);
        const double w0 = G(d.ucf_lsq)[3 * (size_t)e], w1 = G(d.ucf_lsq)[3 * (size_t)e + 1], w2 = G(d.ucf_lsq)[3 * (size_t)e + 2];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double du = Pj[1 + b] - ui[b];
            Gc[b * 3] += du * w0;
            Gc[b * 3 + 1] += du * w1;
            Gc[b * 3 + 2] += du * w2;
        }
    }
    const Soa<double> Gd = soa(d.grad, n, cell);
#pragma unroll
    for (int k = 0; k < 9; ++k) Gd[k] = Gc[k];
}

// Kinetic flux of every face out of its owner, one wave per face: sum over
// the nodes of w (xi.n) psi f_face, psi = (1, xi, |xi|^2 f0 + f1, f1), f_face
// the upwind cell's value inside; on a boundary face the owner's value going
// out and the boundary value coming in, the wall density from this f (zero
// mass flux).  A boundary face also keeps the incoming half-range
// psi-moments of its boundary Maxwellian, w (xi.n) psi M_b over xi.n < 0.
template <typename T, bool DIA>
__global__ __launch_bounds__(256) void k_umac_kin(GSIS_SPAN_ARGS)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    const int f = __builtin_amdgcn_readfirstlane(blk * 4 + (int)(threadIdx.x >> 6));
    if (f >= g.unface) return;
    const int lane = threadIdx.x & 63;
    const int L = G(d.uf_cell)[2 * (size_t)f], R = G(d.uf_cell)[2 * (size_t)f + 1];
    const gptr<const double> fg = G((const double *)d.uf_geo) + 9 * (size_t)f;
    const double n0 = fg[1], n1 = fg[2], n2 = fg[3];
    const size_t nv = (size_t)g.nv;
    const gptr<const T> f0L = (gptr<const T>)d.f0 + (size_t)L * nv;
    const gptr<const T> f1L = DIA ? (gptr<const T>)d.f1 + (size_t)L * nv : f0L;
    const int Rr = R >= 0 ? R : L;
    const gptr<const T> f0R = (gptr<const T>)d.f0 + (size_t)Rr * nv;
    const gptr<const T> f1R = DIA ? (gptr<const T>)d.f1 + (size_t)Rr * nv : f0R;
    const gptr<const double> nt = G((const double *)d.nt64);
    const int bf = R >= 0 ? 0 : -1 - R;
    const int slot = R >= 0 ? 0 : G(d.ubf_slot)[bf];
    const gptr<const double> mb = G((const double *)d.mb64) + (size_t)slot * nv;
    const gptr<const double> mb1 = G((const double *)d.mb1_64) + (size_t)slot * nv;
    double acc[6] = {0, 0, 0, 0, 0, 0}, bin[6] = {0, 0, 0, 0, 0, 0}, out = 0.0, in = 0.0;
    for (int pos = lane; pos < g.nv; pos += 64) {
        const double x0 = nt[4 * (size_t)pos], x1 = nt[4 * (size_t)pos + 1], x2 = nt[4 * (size_t)pos + 2];
        const double w = nt[4 * (size_t)pos + 3];
        const double xn = x0 * n0 + x1 * n1 + x2 * n2;
        if (xn == 0.0) continue;
        double a0, a1;
        bool add = true;
        if (xn > 0.0) {
            a0 = (double)f0L[pos];
            a1 = DIA ? (double)f1L[pos] : 0.0;
            if (R < 0) out += w * xn * a0;
        } else if (R >= 0) {
            a0 = (double)f0R[pos];
            a1 = DIA ? (double)f1R[pos] : 0.0;
        } else {
            a0 = mb[pos];
            a1 = DIA ? mb1[pos] : 0.0;
            in += w * (-xn) * a0;
            add = false;   // into bin: scaled by the wall density once it is known
        }
        const double ww = w * xn, xx = x0 * x0 + x1 * x1 + x2 * x2;
        const double c[6] = {ww * a0, ww * x0 * a0, ww * x1 * a0, ww * x2 * a0, ww * (xx * a0 + a1), ww * a1};
        if (add) {
#pragma unroll
            for (int k = 0; k < 6; ++k) acc[k] += c[k];
        } else {
#pragma unroll
            for (int k = 0; k < 6; ++k) bin[k] += c[k];
        }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] = wave_sum(acc[k]);
    if (R < 0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) bin[k] = wave_sum(bin[k]);
        out = wave_sum(out);
        in = wave_sum(in);
        const double sc = C.bc.kind[slot] == 1 ? C.bc.rho[slot] : out / in;
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[k] += sc * bin[k];
        if (lane < 6) G(d.ubin)[6 * (size_t)bf + lane] = bin[lane];
    }
    if (lane < 6) G(d.uFk)[6 * (size_t)f + lane] = acc[lane];
}

// Interior faces, one thread each: the macroscopic flux of the current W;
// mode 0 keeps F_kin - F as the face's high-order terms, mode 1 stores
// F + HoT and Gamma for the residual.
__global__ __launch_bounds__(256) void k_umac_iflux(GSIS_SPAN_ARGS, int mode, int euler)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    const int f = blk * blockDim.x + threadIdx.x;
    if (f >= g.unface) return;
    const int L = G(d.uf_cell)[2 * (size_t)f], R = G(d.uf_cell)[2 * (size_t)f + 1];
    if (R < 0) return;
    const size_t n = g.ncell;
    double fg[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) fg[k] = G(d.uf_geo)[9 * (size_t)f + k];
    double F[6], Gam;
    uface_flux(g, soa(d.P, n, L), soa(d.P, n, R), soa(d.grad, n, L), soa(d.grad, n, R), fg, euler != 0, F, &Gam);
    if (mode == 0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) G(d.ufix)[6 * (size_t)f + k] = G(d.uFk)[6 * (size_t)f + k] - F[k];
        if (g.species != 1) G(d.ufix)[6 * (size_t)f + 5] = 0.0;
    } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) G(d.uFf)[7 * (size_t)f + k] = F[k] + G(d.ufix)[6 * (size_t)f + k];
        G(d.uFf)[7 * (size_t)f + 6] = Gam;
    }
}

// Stress and heat fluxes of the Grad-13 wall flux at every boundary face's
// cell, one thread per boundary face: the NSF values of the current iterate
// (its least-squares velocity gradient and the gradients of Tt and Tr with the
// same weights) plus the cell's high-order terms.  Mode 0 (at W^{n+1/2})
// forms and keeps those terms, the kinetic stress and heat fluxes of
// f^{n+1/2} minus the NSF values; mode 1 adds the kept terms.  ubsq[12][unbf]
// = (sigma xx yy zz xy xz yz, q, qr).
__global__ __launch_bounds__(256) void k_umac_g13s(GSIS_SPAN_ARGS, int mode)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    const int bf = blk * blockDim.x + threadIdx.x;
    if (bf >= g.unbf) return;
    const size_t n = g.ncell, nb = g.unbf;
    const int cell = G(d.ubf_cell)[bf];
    const Soa<double> P = soa(d.P, n, cell);
    const Soa<double> Gu = soa(d.grad, n, cell);
    double gt[3] = {0, 0, 0}, gr[3] = {0, 0, 0};
    const int first = G(d.ucf_first)[cell], cnt = G(d.ucf_first)[cell + 1] - first;
    for (int k = 0; k < cnt; ++k) {
        const int e = first + k;
        const int j = G(d.ucf_nb)[e];
        if (j < 0) continue;
        const Soa<double> Pj = soa(d.P, n, j);
        const double dt = Pj[4] - P[4], dr = Pj[5] - P[5];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double w = G(d.ucf_lsq)[3 * (size_t)e + c];
            gt[c] += dt * w;
            gr[c] += dr * w;
        }
    }
    const double mu = P[9];
    double G9[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) G9[k] = Gu[k];
    const double div = G9[0] + G9[4] + G9[8];
    double sq[12];
    sq[0] = -mu * (2.0 * G9[0] - (2.0 / 3.0) * div);
    sq[1] = -mu * (2.0 * G9[4] - (2.0 / 3.0) * div);
    sq[2] = -mu * (2.0 * G9[8] - (2.0 / 3.0) * div);
    sq[3] = -mu * (G9[1] + G9[3]);
    sq[4] = -mu * (G9[2] + G9[6]);
    sq[5] = -mu * (G9[5] + G9[7]);
    const bool dia = g.species == 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        sq[6 + c] = -g.kt * mu * gt[c];
        sq[9 + c] = dia ? -g.kr * mu * gr[c] : 0.0;
    }
    const gptr<double> hot = G(d.ubhot);
    if (mode == 0) {
        // cm: sigma at 5..10, q at 11..13, qr at 15..17
        const gptr<const double> m = G((const double *)d.cm) + (size_t)cell * NMOM;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const double kin = k < 9 ? m[5 + k] : (dia ? m[6 + k] : 0.0);
            const double h = kin - sq[k];
            hot[(size_t)k * nb + bf] = h;
            sq[k] += h;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) sq[k] += hot[(size_t)k * nb + bf];
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) G(d.ubsq)[(size_t)k * nb + bf] = sq[k];
}

// Boundary faces, NF to a wave: F_eq of the owner's Maxwellian (outgoing
// half-range sums over the nodes, incoming part the boundary Maxwellian at
// the face's density rule); the wave reads every node's velocity once for
// its NF faces.  Mode 0 keeps F_kin - F_eq(W^{n+1/2}), mode 1 stores fixed
// part + F_eq(W^m) and Gamma.  G13: the same with the outgoing half of the
// owner's Grad-13 distributions of Eq. (G13_VDF) (stress and heat fluxes
// from k_umac_g13s), f0 = M B(c), f1 = (dr/2) Tr f0 + 2 M (qr.c) / (rho Tt).
// Two faces to a wave (tetrahedral block flow, 17k boundary faces x 7788
// nodes, 300 inner iterations: 8 faces 120.3 ms per correction, 4: 106.3,
// 2: 103.7, 1: 116.1; Grad-13 form 4: 140.2, 2: 129.1).
constexpr int UBF = 2, UBF_G13 = 2;

template <int NF, bool G13>
__global__ __launch_bounds__(256) void k_umac_bflux(GSIS_SPAN_ARGS, int mode, int euler)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    constexpr int UBF = NF;
    const int bf0 = __builtin_amdgcn_readfirstlane((blk * 4 + (int)(threadIdx.x >> 6)) * UBF);
    if (bf0 >= g.unbf) return;
    const int lane = threadIdx.x & 63;
    const bool dia = g.species == 1;
    int f[UBF], cell[UBF], slot[UBF];
    double n[UBF][3], u[UBF][3], iT[UBF], s0[UBF], s1[UBF][3], s4[UBF];
    // Grad-13: the bracket's coefficients per face, sigma / (rho Tt^2),
    // 2 q / (rho Tt^2), 2 / (5 Tt), 2 qr / (rho Tt), and the q_r sum
    double sg[G13 ? UBF : 1][6], qv[G13 ? UBF : 1][3], c5[G13 ? UBF : 1], qr[G13 ? UBF : 1][3], sr[G13 ? UBF : 1];
#pragma unroll
    for (int q = 0; q < UBF; ++q) {
        const int bf = min(bf0 + q, g.unbf - 1);
        f[q] = G(d.ubf_face)[bf];
        cell[q] = G(d.ubf_cell)[bf];
        slot[q] = G(d.ubf_slot)[bf];
        const gptr<const double> fg = G((const double *)d.uf_geo) + 9 * (size_t)f[q];
        n[q][0] = fg[1];
        n[q][1] = fg[2];
        n[q][2] = fg[3];
        const Soa<double> P = soa(d.P, (size_t)g.ncell, cell[q]);
        u[q][0] = P[1];
        u[q][1] = P[2];
        u[q][2] = P[3];
        iT[q] = 1.0 / P[4];
        s0[q] = s4[q] = 0.0;
        s1[q][0] = s1[q][1] = s1[q][2] = 0.0;
        if constexpr (G13) {
            const int bf = min(bf0 + q, g.unbf - 1);
            const size_t nb = g.unbf;
            const gptr<const double> b = G((const double *)d.ubsq) + bf;
            const double irT2 = 1.0 / (P[0] * P[4] * P[4]);
            const double cr = 2.0 / (P[0] * P[4]);
#pragma unroll
            for (int k = 0; k < 6; ++k) sg[q][k] = b[(size_t)k * nb] * irT2;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                qv[q][k] = 2.0 * irT2 * b[(size_t)(6 + k) * nb];
                qr[q][k] = dia ? cr * b[(size_t)(9 + k) * nb] : 0.0;
            }
            c5[q] = 2.0 / (5.0 * P[4]);
            sr[q] = 0.0;
        }
    }
    const gptr<const double> nt = G((const double *)d.nt64);
    for (int pos = lane; pos < g.nv; pos += 64) {
        const double x0 = nt[4 * (size_t)pos], x1 = nt[4 * (size_t)pos + 1], x2 = nt[4 * (size_t)pos + 2];
        const double w = nt[4 * (size_t)pos + 3], xx = x0 * x0 + x1 * x1 + x2 * x2;
#pragma unroll
        for (int q = 0; q < UBF; ++q) {
            const double xn = x0 * n[q][0] + x1 * n[q][1] + x2 * n[q][2];
            if (!(xn > 0.0)) continue;
            const double cx = x0 - u[q][0], cy = x1 - u[q][1], cz = x2 - u[q][2];
            if constexpr (G13) {
                const double cc = cx * cx + cy * cy + cz * cz;
                const double e = w * exp_core(fmax(-cc * iT[q], -745.0)) * xn;
                const double scc = sg[q][0] * cx * cx + sg[q][1] * cy * cy + sg[q][2] * cz * cz
                                 + 2.0 * (sg[q][3] * cx * cy + sg[q][4] * cx * cz + sg[q][5] * cy * cz);
                const double qc = qv[q][0] * cx + qv[q][1] * cy + qv[q][2] * cz;
                const double ex = e * (1.0 + scc + qc * (c5[q] * cc - 1.0));
                s0[q] += ex;
                s1[q][0] += ex * x0;
                s1[q][1] += ex * x1;
                s1[q][2] += ex * x2;
                s4[q] += ex * xx;
                sr[q] += e * (qr[q][0] * cx + qr[q][1] * cy + qr[q][2] * cz);
            } else {
                const double ex = w * exp_core(fmax(-(cx * cx + cy * cy + cz * cz) * iT[q], -745.0)) * xn;
                s0[q] += ex;
                s1[q][0] += ex * x0;
                s1[q][1] += ex * x1;
                s1[q][2] += ex * x2;
                s4[q] += ex * xx;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < UBF; ++q) {
        s0[q] = wave_sum(s0[q]);
#pragma unroll
        for (int k = 0; k < 3; ++k) s1[q][k] = wave_sum(s1[q][k]);
        s4[q] = wave_sum(s4[q]);
        if constexpr (G13) sr[q] = wave_sum(sr[q]);
    }
    // lane q finishes face q
#pragma unroll
    for (int q = 0; q < UBF; ++q) {
        if (lane != q || bf0 + q >= g.unbf) continue;
        const Soa<double> P = soa(d.P, (size_t)g.ncell, cell[q]);
        const double rho = P[0], T = P[4];
        const double piT = PI * T, K = rho / (piT * sqrt(piT));
        const double h1 = g.species == 1 ? 0.5 * g.dr * P[5] : 0.0;
        double out[6];
        out[0] = K * s0[q];
#pragma unroll
        for (int k = 0; k < 3; ++k) out[1 + k] = K * s1[q][k];
        if constexpr (G13) {
            const double f1 = dia ? K * (h1 * s0[q] + sr[q]) : 0.0;
            out[4] = K * s4[q] + f1;
            out[5] = f1;
        } else {
            out[4] = K * s4[q] + h1 * out[0];
            out[5] = h1 * out[0];
        }
        const int bf = bf0 + q;
        const gptr<const double> bin = G((const double *)d.ubin) + 6 * (size_t)bf;
        const double sc = C.bc.kind[slot[q]] == 1 ? C.bc.rho[slot[q]] : out[0] / (-bin[0]);
        double Fe[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) Fe[k] = out[k] + sc * bin[k];
        const size_t ff = f[q];
        if (mode == 0) {
#pragma unroll
            for (int k = 0; k < 6; ++k) G(d.ufix)[6 * ff + k] = G(d.uFk)[6 * ff + k] - Fe[k];
        } else {
#pragma unroll
            for (int k = 0; k < 6; ++k) G(d.uFf)[7 * ff + k] = G(d.ufix)[6 * ff + k] + Fe[k];
            const double un = u[q][0] * n[q][0] + u[q][1] * n[q][1] + u[q][2] * n[q][2];
            G(d.uFf)[7 * ff + 6] = fabs(un) + P[8] + (euler ? 0.0 : g.Cd * P[9] / (rho * G(d.uf_geo)[9 * ff + 4]));
        }
    }
}

// Residual and diagonal of every cell from the face fluxes (S / V per face,
// the sign of the owner's side), the rotational relaxation on the Er row; one
// atomic max of D per wave into the slot's partials.
__global__ __launch_bounds__(256) void k_umac_res(GSIS_SPAN_ARGS, int slot, int euler)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    const int cell = blk * blockDim.x + threadIdx.x;
    double D = 0.0;
    if (cell < g.ncell) {
        const size_t n = g.ncell;
        const Soa<double> P = soa(d.P, n, cell);
        double res[6] = {0, 0, 0, 0, 0, 0}, sumG = 0.0;
        const double iV = 1.0 / G(d.uvol)[cell];
        const int first = G(d.ucf_first)[cell], cnt = G(d.ucf_first)[cell + 1] - first;
        for (int k = 0; k < cnt; ++k) {
            const int fs = G(d.ucf_face)[first + k], f = fs >> 1;
            const double sv = G(d.uf_geo)[9 * (size_t)f] * iV, sg = (fs & 1) ? -1.0 : 1.0;
            const gptr<const double> o = G((const double *)d.uFf) + 7 * (size_t)f;
#pragma unroll
            for (int q = 0; q < 6; ++q) res[q] -= sg * o[q] * sv;
            sumG += o[6] * sv;
        }
        if (g.species != 1) res[5] = 0.0;
        const double invtau = P[10];
        if (g.species == 1) {
            const double T = (3.0 * P[4] + g.dr * P[5]) / (3.0 + g.dr);
            res[5] += 0.5 * g.dr * P[0] * (T - P[5]) * invtau / g.Zr;
        }
        const double umag = sqrt(P[1] * P[1] + P[2] * P[2] + P[3] * P[3]);
        const double vis = euler ? 0.0 : g.Cd * P[9] / (P[0] * g.uhmin);
        const double idt = (umag + P[8] + vis) / (g.macro_cfl * g.uhmin);
        D = idt + 0.5 * sumG;
        const Soa<double> r = soa(d.R, n, cell);
#pragma unroll
        for (int q = 0; q < 6; ++q) r[q] = res[q];
        G(d.Src)[cell] = g.species == 1 ? invtau / g.Zr : 0.0;
        if (!(D > 0.0 && isfinite(D))) {
            atomicOr(d.errflag, 2);
            D = 0.0;
        }
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) D = fmax(D, __shfl_xor(D, m, 64));
    if ((threadIdx.x & 63) == 0 && D > 0.0)
        atomicMax(&d.dmax[(size_t)(slot * DSLOT + ((blk * 4 + (int)(threadIdx.x >> 6)) & (DSLOT - 1))) * DSTRIDE],
                  (unsigned long long)__double_as_longlong(D));
}

// W += R / D* (the Er row with its relaxation on the diagonal) and the new
// prims; block 0 clears the partials of the other slot (the previous
// iteration's).
__global__ __launch_bounds__(256) void k_umac_advance(GSIS_SPAN_ARGS, int slot)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    double Dm = __longlong_as_double((long long)G(d.dmax)[(size_t)(slot * DSLOT + (threadIdx.x & (DSLOT - 1))) * DSTRIDE]);
#pragma unroll
    for (int m = 1; m < DSLOT; m <<= 1) Dm = fmax(Dm, __shfl_xor(Dm, m, 64));
    if (blk == 0 && (int)threadIdx.x < DSLOT) G(d.dmax)[(size_t)((slot ^ 1) * DSLOT + threadIdx.x) * DSTRIDE] = 0ull;
    const int cell = blk * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    const size_t n = g.ncell;
    const double iDm = 1.0 / Dm;
    const Soa<double> W = soa(d.W, n, cell);
    const Soa<double> r = soa(d.R, n, cell);
    double Wn[6];
#pragma unroll
    for (int k = 0; k < 5; ++k) Wn[k] = W[k] + r[k] * iDm;
    Wn[5] = g.species == 1 ? W[5] + r[5] / (Dm + G(d.Src)[cell]) : W[5];
#pragma unroll
    for (int k = 0; k < 6; ++k) W[k] = Wn[k];
    prim_from_W(g, Wn, soa(d.P, n, cell));
}

// Euler steps: no high-order terms, the boundary flux of the iterate's own
// Maxwellian -- every fixed part zero.
__global__ __launch_bounds__(256) void k_umac_nofix(GSIS_SPAN_ARGS)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const int i = blk * blockDim.x + threadIdx.x;
    if (i < 6 * C.g.unface) G(C.d.ufix)[i] = 0.0;
}

hipError_t launch_umacro(const Target &t, int iters, hipStream_t s, int euler)
{
    const Geo &g = t.host->g;
    const Span sp{t.cases, nullptr};
    const dim3 cells((g.ncell + 255) / 256), faces((g.unface + 255) / 256);
    const dim3 fwaves((g.unface + 3) / 4), bwaves(((std::max(g.unbf, 1) + UBF - 1) / UBF + 3) / 4);
    const dim3 gwaves(((std::max(g.unbf, 1) + UBF_G13 - 1) / UBF_G13 + 3) / 4), bthreads((std::max(g.unbf, 1) + 255) / 256);
    // the Grad-13 wall flux: its stress and heat fluxes first, then its flux
    const bool g13 = t.g13 && !euler;
    auto bflux = [&](int mode) {
        if (g13) {
            hipLaunchKernelGGL(k_umac_g13s, bthreads, dim3(256), 0, s, GSIS_SPAN(sp), mode);
            hipLaunchKernelGGL((k_umac_bflux<UBF_G13, true>), gwaves, dim3(256), 0, s, GSIS_SPAN(sp), mode, euler);
        } else {
            hipLaunchKernelGGL((k_umac_bflux<UBF, false>), bwaves, dim3(256), 0, s, GSIS_SPAN(sp), mode, euler);
        }
    };
    hipLaunchKernelGGL(k_mac_reset, dim3(1), dim3(64), 0, s, GSIS_SPAN(sp));
    hipLaunchKernelGGL(k_mac_init, dim3(t.nblk[K_CELL128]), dim3(128), 0, s, GSIS_SPAN(sp));
    hipLaunchKernelGGL(k_umac_grad, cells, dim3(256), 0, s, GSIS_SPAN(sp));
    // the kinetic face fluxes, and the boundary Maxwellians' incoming moments the boundary fluxes need
    if (t.fp32) {
        if (t.dia) hipLaunchKernelGGL((k_umac_kin<float, true>), fwaves, dim3(256), 0, s, GSIS_SPAN(sp));
        else hipLaunchKernelGGL((k_umac_kin<float, false>), fwaves, dim3(256), 0, s, GSIS_SPAN(sp));
    } else {
        if (t.dia) hipLaunchKernelGGL((k_umac_kin<double, true>), fwaves, dim3(256), 0, s, GSIS_SPAN(sp));
        else hipLaunchKernelGGL((k_umac_kin<double, false>), fwaves, dim3(256), 0, s, GSIS_SPAN(sp));
    }
    if (euler) {
        hipLaunchKernelGGL(k_umac_nofix, dim3((6 * g.unface + 255) / 256), dim3(256), 0, s, GSIS_SPAN(sp));
    } else {
        hipLaunchKernelGGL(k_umac_iflux, faces, dim3(256), 0, s, GSIS_SPAN(sp), 0, 0);
        if (g.unbf > 0) bflux(0);
    }
    for (int it = 0; it < iters; ++it) {
        const int slot = it & 1;
        if (it > 0) hipLaunchKernelGGL(k_umac_grad, cells, dim3(256), 0, s, GSIS_SPAN(sp));
        hipLaunchKernelGGL(k_umac_iflux, faces, dim3(256), 0, s, GSIS_SPAN(sp), 1, euler);
        if (g.unbf > 0) bflux(1);
        hipLaunchKernelGGL(k_umac_res, cells, dim3(256), 0, s, GSIS_SPAN(sp), slot, euler);
        hipLaunchKernelGGL(k_umac_advance, cells, dim3(256), 0, s, GSIS_SPAN(sp), slot);
    }
    hipLaunchKernelGGL(k_mac_final, dim3(t.nblk[K_CELL128]), dim3(128), 0, s, GSIS_SPAN(sp));
    return hipGetLastError();
}

// blocks one case needs for each launch shape
int kind_blocks(const Geo &g, Kind k)
{
    switch (k) {
    case K_CELL64: return (g.ncell + 63) / 64;
    case K_CELL128: return (g.ncell + 127) / 128;
    case K_CELL256: return (g.ncell + 255) / 256;
    case K_CELL1: return g.ncell;
    case K_FACE256: return (g.nface + 255) / 256;
    case K_FACE8: return face_blocks(g);
    case K_GRAD: return grad_blocks(g) + face_blocks(g);
    case K_RES: return (g.ncell + RES_CELLS - 1) / RES_CELLS;
    case K_CASE: return 1;
    default: return 0;
    }
}

}  // namespace gsis

// Per-cell parameters of the relaxation target and per-face boundary
// densities, FP64.
//
// The reference distribution of Sec. 2.2 is written around the cell's
// Maxwellian shape E = exp(-|c|^2 / T), c = xi - u, so the sweep evaluates
//   monatomic: g / tau = A E [P0 + l.c + l4 |c|^2 + (qp.c)(|c|^2/T - 5/2)],
//   diatomic:  the Rykov mixture (1 - 1/Z) g_t + g_r / Z of the four
//              components, two shapes (Tt and T), one exponential each,
// with one exponential per shape and node.  l, l4, P0 - 1 are the
// conservative correction: they make the discrete moments (1, xi, |xi|^2) of
// each component equal their continuous values exactly.  On the tensor grid
// the 5x5 Gram matrix sum w phi phi^T M and the Shakhov term's moments factor
// into 1-D sums C_a(p) = sum_k w_k c^p exp(-c^2/T), p <= 5, so the correction
// costs O(n per axis) per cell.
#include "gsis_common.h"
#include "gsis_launch.h"

namespace gsis {

__device__ void axis_central(const double *xi, const double *w, int n, double u, double T, double C[6])
{
    for (int p = 0; p < 6; ++p) C[p] = 0.0;
    for (int k = 0; k < n; ++k) {
        double c = xi[k] - u;
        double e = w[k] * exp(-c * c / T);
        C[0] += e;
        e *= c; C[1] += e;
        e *= c; C[2] += e;
        e *= c; C[3] += e;
        e *= c; C[4] += e;
        e *= c; C[5] += e;
    }
}

struct Sep {
    double C[3][6];
    __device__ double m(int p, int q, int r) const { return C[0][p] * C[1][q] * C[2][r]; }
};

// phi = (1, c_x, c_y, c_z, |c|^2) as monomial lists
__device__ __forceinline__ int phi_terms(int i, int t[3][3])
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) t[a][b] = 0;
    if (i == 0) return 1;
    if (i <= 3) { t[0][i - 1] = 1; return 1; }
    t[0][0] = 2; t[1][1] = 2; t[2][2] = 2;
    return 3;
}

// Gram G_ij = sum phi_i phi_j E and Shakhov moments bS_i = sum phi_i E [1 + (qp.c)(|c|^2 kT - 5/2)],
// both without the prefactor rho (pi T)^{-3/2}.
__device__ void gram_and_shakhov(const Sep &S, const double qp[3], double kT, double G[25], double bS[5])
{
    int ti[3][3], tj[3][3];
    for (int i = 0; i < 5; ++i) {
        int ni = phi_terms(i, ti);
        for (int j = 0; j < 5; ++j) {
            int nj = phi_terms(j, tj);
            double s = 0.0;
            for (int a = 0; a < ni; ++a)
                for (int b = 0; b < nj; ++b) s += S.m(ti[a][0] + tj[b][0], ti[a][1] + tj[b][1], ti[a][2] + tj[b][2]);
            G[i * 5 + j] = s;
        }
        double s = 0.0;
        for (int a = 0; a < ni; ++a) {
            const int *e = ti[a];
            s += S.m(e[0], e[1], e[2]);
            for (int ax = 0; ax < 3; ++ax) {
                int f[3] = {e[0], e[1], e[2]};
                f[ax] += 1;
                double cube = S.m(f[0] + 2, f[1], f[2]) + S.m(f[0], f[1] + 2, f[2]) + S.m(f[0], f[1], f[2] + 2);
                s += qp[ax] * (kT * cube - 2.5 * S.m(f[0], f[1], f[2]));
            }
        }
        bS[i] = s;
    }
}

// Dense 5x5 solve with partial pivoting; a pivot below 1e-12 of the largest
// entry counts as zero (singular: false).  On a velocity grid where 1, xi and
// |xi|^2 are linearly dependent (two nodes +-a per axis) the conservative
// correction is singular and is then not applied.
__device__ bool solve5(double *A, double *b)
{
    double amax = 0.0;
    for (int i = 0; i < 25; ++i) amax = fmax(amax, fabs(A[i]));
    for (int k = 0; k < 5; ++k) {
        int piv = k;
        for (int i = k + 1; i < 5; ++i)
            if (fabs(A[i * 5 + k]) > fabs(A[piv * 5 + k])) piv = i;
        if (!(fabs(A[piv * 5 + k]) > 1e-12 * amax)) return false;
        if (piv != k) {
            for (int j = 0; j < 5; ++j) { double t = A[k * 5 + j]; A[k * 5 + j] = A[piv * 5 + j]; A[piv * 5 + j] = t; }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int i = k + 1; i < 5; ++i) {
            double f = A[i * 5 + k] / A[k * 5 + k];
            for (int j = k; j < 5; ++j) A[i * 5 + j] -= f * A[k * 5 + j];
            b[i] -= f * b[k];
        }
    }
    for (int k = 4; k >= 0; --k) {
        double t = b[k];
        for (int j = k + 1; j < 5; ++j) t -= A[k * 5 + j] * b[j];
        b[k] = t / A[k * 5 + k];
    }
    return true;
}

// Correction lambda (c-basis) of one component with shape rho (pi T)^{-3/2} E:
// K G lambda = target - K bS, target = (rho, 0, 0, 0, 1.5 rho T).
__device__ void correction(const Sep &S, double K, double rho, double T, const double qp[3], double kT,
                           bool conservative, double lam[5], double bS[5])
{
    double G[25];
    gram_and_shakhov(S, qp, kT, G, bS);
    for (int i = 0; i < 5; ++i) lam[i] = 0.0;
    if (!conservative) return;
    double tgt[5] = {rho, 0.0, 0.0, 0.0, 1.5 * rho * T};
    for (int i = 0; i < 25; ++i) G[i] *= K;
    for (int i = 0; i < 5; ++i) lam[i] = tgt[i] - K * bS[i];
    if (!solve5(G, lam))
        for (int i = 0; i < 5; ++i) lam[i] = 0.0;
}

// Parameter layout (NPAR doubles per cell):
//  monatomic: 0-2 u, 3 1/Tt, 4 A = rho (pi Tt)^{-3/2} / tau, 5 P0 = 1 + l0, 6-8 l_c, 9 l4,
//             10-12 qp = (4/15) q / (rho Tt^2), 13 1/tau
//  diatomic:  0-2 u, 3 1/Tt, 4 1/T, 5 At, 6 Ar (shape prefactors times (1-1/Z)/tau and 1/(Z tau)),
//             7 P0t, 8-10 l_t, 11 l4t, 12-14 qp_t, 15 P0r, 16-18 l_r, 19 l4r, 20-22 qp_r,
//             23 ht = (dr/2) Tr, 24-26 2 qr / (rho Tt), 27 nu_t,
//             28 hr = (dr/2) T, 29-31 2 q1 / (rho T), 32 nu_r, 33 1/tau
__global__ __launch_bounds__(64) void k_params(GSIS_SPAN_ARGS)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    int cell = blk * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    double *p = d.par + (size_t)cell * NPAR;
    float *pf = d.parf + (size_t)cell * NPAR;
    if (!d.cflag[cell]) {
        for (int k = 0; k < NPAR; ++k) { p[k] = 0.0; pf[k] = 0.0f; }
        return;
    }
    const double *m = d.cm + (size_t)cell * NMOM;
    double rho = m[0], u[3] = {m[1], m[2], m[3]}, Tt = m[4];
    double q[3] = {m[11], m[12], m[13]};
    double invtau = g.delta * rho * pow(Tt, 1.0 - g.omega);
    if (!(rho > 0.0) || !(Tt > 0.0) || !isfinite(invtau)) atomicOr(d.errflag, 1);
    for (int k = 0; k < NPAR; ++k) p[k] = 0.0;
    bool cons = g.conservative != 0;
    if (g.species == 0) {
        Sep S;
        for (int a = 0; a < 3; ++a) axis_central(d.xi64[a], d.w64[a], g.n1[a], u[a], Tt, S.C[a]);
        double K = rho * pow(PI * Tt, -1.5);
        double kT = 1.0 / Tt;
        double qp[3];
        for (int a = 0; a < 3; ++a) qp[a] = (4.0 / 15.0) * q[a] / (rho * Tt * Tt);
        double lam[5], bS[5];
        correction(S, K, rho, Tt, qp, kT, cons, lam, bS);
        p[0] = u[0]; p[1] = u[1]; p[2] = u[2];
        p[3] = kT;
        p[4] = K * invtau;
        p[5] = 1.0 + lam[0];
        p[6] = lam[1]; p[7] = lam[2]; p[8] = lam[3];
        p[9] = lam[4];
        p[10] = qp[0]; p[11] = qp[1]; p[12] = qp[2];
        p[13] = invtau;
    } else {
        double Tr = m[14], qr[3] = {m[15], m[16], m[17]};
        double dr = g.dr, Z = g.Zr;
        double T = (3.0 * Tt + dr * Tr) / (3.0 + dr);
        double Att = g.A[0], Atr = g.A[1], Art = g.A[2], Arr = g.A[3];
        double q0[3], q1[3];
        for (int a = 0; a < 3; ++a) {
            q0[a] = ((2.0 - 3.0 * Att) * Z + 1.0) * q[a] + (-3.0 * Atr * Z) * qr[a];
            q1[a] = (-Art * Z) * q[a] + (-Arr * Z + 1.0) * qr[a];
        }
        Sep St, Sr;
        for (int a = 0; a < 3; ++a) {
            axis_central(d.xi64[a], d.w64[a], g.n1[a], u[a], Tt, St.C[a]);
            axis_central(d.xi64[a], d.w64[a], g.n1[a], u[a], T, Sr.C[a]);
        }
        double Kt = rho * pow(PI * Tt, -1.5), Kr = rho * pow(PI * T, -1.5);
        double kTt = 1.0 / Tt, kT = 1.0 / T;
        double qpt[3], qpr[3];
        for (int a = 0; a < 3; ++a) {
            qpt[a] = (4.0 / 15.0) * q[a] / (rho * Tt * Tt);
            qpr[a] = (4.0 / 15.0) * q0[a] / (rho * T * T);
        }
        double lt[5], lr[5], bSt[5], bSr[5];
        correction(St, Kt, rho, Tt, qpt, kTt, cons, lt, bSt);
        correction(Sr, Kr, rho, T, qpr, kT, cons, lr, bSr);
        double ht = 0.5 * dr * Tr, hr = 0.5 * dr * T;
        double qrt[3], q1r[3];
        for (int a = 0; a < 3; ++a) {
            qrt[a] = 2.0 * qr[a] / (rho * Tt);
            q1r[a] = 2.0 * q1[a] / (rho * T);
        }
        // sum_w g_1t = ht Kt bSt[0] + Kt qrt.m(e_a); the correction nu Kt E matches (dr/2) rho Tr
        double s1t = ht * Kt * bSt[0] + Kt * (qrt[0] * St.m(1, 0, 0) + qrt[1] * St.m(0, 1, 0) + qrt[2] * St.m(0, 0, 1));
        double s1r = hr * Kr * bSr[0] + Kr * (q1r[0] * Sr.m(1, 0, 0) + q1r[1] * Sr.m(0, 1, 0) + q1r[2] * Sr.m(0, 0, 1));
        double nut = cons ? (0.5 * dr * rho * Tr - s1t) / (Kt * St.m(0, 0, 0)) : 0.0;
        double nur = cons ? (0.5 * dr * rho * T - s1r) / (Kr * Sr.m(0, 0, 0)) : 0.0;
        double iz = 1.0 / Z;
        p[0] = u[0]; p[1] = u[1]; p[2] = u[2];
        p[3] = kTt;
        p[4] = kT;
        p[5] = (1.0 - iz) * Kt * invtau;
        p[6] = iz * Kr * invtau;
        p[7] = 1.0 + lt[0];
        p[8] = lt[1]; p[9] = lt[2]; p[10] = lt[3];
        p[11] = lt[4];
        p[12] = qpt[0]; p[13] = qpt[1]; p[14] = qpt[2];
        p[15] = 1.0 + lr[0];
        p[16] = lr[1]; p[17] = lr[2]; p[18] = lr[3];
        p[19] = lr[4];
        p[20] = qpr[0]; p[21] = qpr[1]; p[22] = qpr[2];
        p[23] = ht;
        p[24] = qrt[0]; p[25] = qrt[1]; p[26] = qrt[2];
        p[27] = nut;
        p[28] = hr;
        p[29] = q1r[0]; p[30] = q1r[1]; p[31] = q1r[2];
        p[32] = nur;
        p[33] = invtau;
    }
    for (int k = 0; k < NPAR; ++k) pf[k] = (float)p[k];
}

// Incoming density scale of every boundary face.  Diffuse wall: the outgoing
// mass flux of the cell's current state (from its octant sums) over the
// incoming flux of M(1, u_w, T_w), so the discrete wall mass flux is zero;
// inflow: the prescribed density.
__global__ __launch_bounds__(256) void k_face_scale(GSIS_SPAN_ARGS)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const BcInfo &bc = C.bc;
    const Dev &d = C.d;
    int f = blk * blockDim.x + threadIdx.x;
    if (f >= g.nface) return;
    int cell = d.face_cell[f], dir = d.face_dir[f], b = d.face_bc[f];
    double sc;
    if (bc.kind[b] == 1) {
        sc = bc.rho[b];
    } else {
        int a = dir / 2;
        int neg = (dir & 1) ? 0 : 1;   // outgoing nodes: xi_a > 0 on a + face, xi_a < 0 on a - face
        double out = 0.0;
        for (int o = 0; o < 8; ++o)
            if (((o >> a) & 1) == neg) out += d.mom8[((size_t)cell * 8 + o) * NRS + 1 + a];
        if (neg) out = -out;
        sc = out / (-d.inpsi[(b * 6 + dir) * 6 + 0]);
    }
    d.fscale[f] = sc;
    d.fscalef[f] = (float)sc;
    d.cfs64[(size_t)cell * 6 + dir] = sc;
    d.cfs32[(size_t)cell * 6 + dir] = (float)sc;
}

hipError_t launch_params(const Target &t, hipStream_t s)
{
    hipLaunchKernelGGL(k_params, dim3(t.nblk[K_CELL64]), dim3(64), 0, s, GSIS_SPAN(t.span(K_CELL64)));
    return hipGetLastError();
}

hipError_t launch_face_scale(const Target &t, hipStream_t s)
{
    if (t.nblk[K_FACE256] > 0)
        hipLaunchKernelGGL(k_face_scale, dim3(t.nblk[K_FACE256]), dim3(256), 0, s, GSIS_SPAN(t.span(K_FACE256)));
    return hipGetLastError();
}

}  // namespace gsis

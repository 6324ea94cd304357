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
// costs O(n per axis) per cell.  On a node list (a refined or unstructured
// velocity mesh, Sec. 3.1) nothing factors: the Gram matrix and the Shakhov
// moments are summed over the nodes directly, one wave per cell.
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

// Gram matrix and Shakhov moments of one shape on the velocity grid (without
// the prefactor): G_ij = sum w phi_i phi_j E, bS_i = sum w phi_i E [1 +
// (qp.c)(|c|^2 kT - 5/2)].  G_00 = sum w E and G_0a = sum w c_a E.
struct ShapeSums {
    double G[25], bS[5];
};

// Correction lambda (c-basis) of one component with shape rho (pi T)^{-3/2} E:
// K G lambda = target - K bS, target = (rho, 0, 0, 0, 1.5 rho T).
__device__ void correction(const ShapeSums &S, double K, double rho, double T, bool conservative, double lam[5])
{
    for (int i = 0; i < 5; ++i) lam[i] = 0.0;
    if (!conservative) return;
    double G[25];
    for (int i = 0; i < 25; ++i) G[i] = K * S.G[i];
    double tgt[5] = {rho, 0.0, 0.0, 0.0, 1.5 * rho * T};
    for (int i = 0; i < 5; ++i) lam[i] = tgt[i] - K * S.bS[i];
    if (!solve5(G, lam))
        for (int i = 0; i < 5; ++i) lam[i] = 0.0;
}

// Moments of one cell and what follows from them alone.
struct CellState {
    double rho, u[3], Tt, q[3], invtau;
    double qpt[3];          // (4/15) q / (rho Tt^2), the Shakhov vector of the Tt shape
    double Tr, qr[3], T;    // diatomic; T = (3 Tt + dr Tr) / (3 + dr)
    double q1[3], qpr[3];   // diatomic: q1 = -A_rt Z q + (1 - A_rr Z) qr; qpr of the T shape
};

// false for a solid cell (its parameters are zeroed)
__device__ bool cell_state(const Geo &g, const Dev &d, int cell, CellState &st)
{
    double *p = d.par + (size_t)cell * NPAR;
    float *pf = d.parf + (size_t)cell * NPAR;
    if (!d.cflag[cell]) {
        for (int k = 0; k < NPAR; ++k) { p[k] = 0.0; pf[k] = 0.0f; }
        return false;
    }
    const double *m = d.cm + (size_t)cell * NMOM;
    st.rho = m[0];
    for (int a = 0; a < 3; ++a) { st.u[a] = m[1 + a]; st.q[a] = m[11 + a]; }
    st.Tt = m[4];
    st.invtau = g.delta * st.rho * pow(st.Tt, 1.0 - g.omega);
    if (!(st.rho > 0.0) || !(st.Tt > 0.0) || !isfinite(st.invtau)) atomicOr(d.errflag, 1);
    for (int a = 0; a < 3; ++a) st.qpt[a] = (4.0 / 15.0) * st.q[a] / (st.rho * st.Tt * st.Tt);
    st.Tr = st.T = st.Tt;
    for (int a = 0; a < 3; ++a) st.qr[a] = st.q1[a] = st.qpr[a] = 0.0;
    if (g.species != 0) {
        st.Tr = m[14];
        for (int a = 0; a < 3; ++a) st.qr[a] = m[15 + a];
        const double T = (3.0 * st.Tt + g.dr * st.Tr) / (3.0 + g.dr);
        st.T = T;
        const double Z = g.Zr, Att = g.A[0], Atr = g.A[1], Art = g.A[2], Arr = g.A[3];
        for (int a = 0; a < 3; ++a) {
            const double q0 = ((2.0 - 3.0 * Att) * Z + 1.0) * st.q[a] + (-3.0 * Atr * Z) * st.qr[a];
            st.q1[a] = (-Art * Z) * st.q[a] + (-Arr * Z + 1.0) * st.qr[a];
            st.qpr[a] = (4.0 / 15.0) * q0 / (st.rho * T * T);
        }
    }
    return true;
}

// Parameter layout (NPAR doubles per cell):
//  monatomic: 0-2 u, 3 1/Tt, 4 A = rho (pi Tt)^{-3/2} / tau, 5 P0 = 1 + l0, 6-8 l_c, 9 l4,
//             10-12 qp = (4/15) q / (rho Tt^2), 13 1/tau
//  diatomic:  0-2 u, 3 1/Tt, 4 1/T, 5 At, 6 Ar (shape prefactors times (1-1/Z)/tau and 1/(Z tau)),
//             7 P0t, 8-10 l_t, 11 l4t, 12-14 qp_t, 15 P0r, 16-18 l_r, 19 l4r, 20-22 qp_r,
//             23 ht = (dr/2) Tr, 24-26 2 qr / (rho Tt), 27 nu_t,
//             28 hr = (dr/2) T, 29-31 2 q1 / (rho T), 32 nu_r, 33 1/tau
// Et: the sums of the shape exp(-|c|^2/Tt) with qp_t on the velocity grid;
// Er: of exp(-|c|^2/T) with qp_r (diatomic only).
__device__ void cell_params(const Geo &g, const Dev &d, int cell, const CellState &st, const ShapeSums &Et,
                            const ShapeSums &Er)
{
    double *p = d.par + (size_t)cell * NPAR;
    float *pf = d.parf + (size_t)cell * NPAR;
    const double rho = st.rho, Tt = st.Tt, invtau = st.invtau;
    const double *u = st.u;
    for (int k = 0; k < NPAR; ++k) p[k] = 0.0;
    bool cons = g.conservative != 0;
    if (g.species == 0) {
        double K = rho * pow(PI * Tt, -1.5);
        double lam[5];
        correction(Et, K, rho, Tt, cons, lam);
        p[0] = u[0]; p[1] = u[1]; p[2] = u[2];
        p[3] = 1.0 / Tt;
        p[4] = K * invtau;
        p[5] = 1.0 + lam[0];
        p[6] = lam[1]; p[7] = lam[2]; p[8] = lam[3];
        p[9] = lam[4];
        p[10] = st.qpt[0]; p[11] = st.qpt[1]; p[12] = st.qpt[2];
        p[13] = invtau;
    } else {
        const double Tr = st.Tr, T = st.T, *qr = st.qr, *q1 = st.q1;
        double dr = g.dr, Z = g.Zr;
        double Kt = rho * pow(PI * Tt, -1.5), Kr = rho * pow(PI * T, -1.5);
        double lt[5], lr[5];
        correction(Et, Kt, rho, Tt, cons, lt);
        correction(Er, Kr, rho, T, cons, lr);
        double ht = 0.5 * dr * Tr, hr = 0.5 * dr * T;
        double qrt[3], q1r[3];
        for (int a = 0; a < 3; ++a) {
            qrt[a] = 2.0 * qr[a] / (rho * Tt);
            q1r[a] = 2.0 * q1[a] / (rho * T);
        }
        // sum_w g_1t = ht Kt bSt[0] + Kt qrt.(sum w c E); the correction nu Kt E matches (dr/2) rho Tr
        double s1t = ht * Kt * Et.bS[0] + Kt * (qrt[0] * Et.G[1] + qrt[1] * Et.G[2] + qrt[2] * Et.G[3]);
        double s1r = hr * Kr * Er.bS[0] + Kr * (q1r[0] * Er.G[1] + q1r[1] * Er.G[2] + q1r[2] * Er.G[3]);
        double nut = cons ? (0.5 * dr * rho * Tr - s1t) / (Kt * Et.G[0]) : 0.0;
        double nur = cons ? (0.5 * dr * rho * T - s1r) / (Kr * Er.G[0]) : 0.0;
        double iz = 1.0 / Z;
        p[0] = u[0]; p[1] = u[1]; p[2] = u[2];
        p[3] = 1.0 / Tt;
        p[4] = 1.0 / T;
        p[5] = (1.0 - iz) * Kt * invtau;
        p[6] = iz * Kr * invtau;
        p[7] = 1.0 + lt[0];
        p[8] = lt[1]; p[9] = lt[2]; p[10] = lt[3];
        p[11] = lt[4];
        p[12] = st.qpt[0]; p[13] = st.qpt[1]; p[14] = st.qpt[2];
        p[15] = 1.0 + lr[0];
        p[16] = lr[1]; p[17] = lr[2]; p[18] = lr[3];
        p[19] = lr[4];
        p[20] = st.qpr[0]; p[21] = st.qpr[1]; p[22] = st.qpr[2];
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

// Tensor grid: one thread per cell, the shape sums from 1-D sums.
__global__ __launch_bounds__(64) void k_params(GSIS_SPAN_ARGS)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    int cell = blk * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    CellState st;
    if (!cell_state(g, d, cell, st)) return;
    ShapeSums Et, Er;
    {
        Sep S;
        for (int a = 0; a < 3; ++a) axis_central(d.xi64[a], d.w64[a], g.n1[a], st.u[a], st.Tt, S.C[a]);
        gram_and_shakhov(S, st.qpt, 1.0 / st.Tt, Et.G, Et.bS);
    }
    if (g.species != 0) {
        Sep S;
        for (int a = 0; a < 3; ++a) axis_central(d.xi64[a], d.w64[a], g.n1[a], st.u[a], st.T, S.C[a]);
        gram_and_shakhov(S, st.qpr, 1.0 / st.T, Er.G, Er.bS);
    }
    cell_params(g, d, cell, st, Et, g.species != 0 ? Er : Et);
}

// Node list, in two kernels.  k_params_list_sums: one wave per cell; each
// lane sums, over the nodes 64 apart (two nodes per step, two independent
// exponentials in flight), the 15 distinct Gram entries and the 5 Shakhov
// moments of each shape directly; the partial sums go through LDS, where lane
// k adds the 64 partials of sum k in lane order, into d.lsum.
// k_params_list_finish: one thread per cell builds the parameters from them
// (kept apart so the summing kernel's register count, and so its occupancy,
// does not carry the dense solves).
template <int NSH>
__global__ __launch_bounds__(64) void k_params_list_sums(GSIS_SPAN_ARGS)
{
    constexpr int NS = LSUM_SHAPE, NA = NS * NSH;
    __shared__ double part[NA][65];
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    const int cell = blk;
    const int lane = threadIdx.x;
    CellState st;
    if (!cell_state(g, d, cell, st)) return;   // uniform over the block
    const gptr<const double> nt = (gptr<const double>)d.nt64;
    double iT[NSH], qp[NSH][3];
#pragma unroll
    for (int sh = 0; sh < NSH; ++sh) {
        iT[sh] = 1.0 / (sh ? st.T : st.Tt);
#pragma unroll
        for (int a = 0; a < 3; ++a) qp[sh][a] = sh ? st.qpr[a] : st.qpt[a];
    }
    double acc[NA];
#pragma unroll
    for (int k = 0; k < NA; ++k) acc[k] = 0.0;
    const int nv = g.nv;
    for (int l0 = 0; l0 < nv; l0 += 128) {
        double t[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int l = l0 + h * 64 + lane;
            const gptr<const double> tp = nt + 4 * (size_t)min(l, nv - 1);
#pragma unroll
            for (int q = 0; q < 4; ++q) t[h][q] = tp[q];
            if (l >= nv) t[h][3] = 0.0;   // a repeated last node counts zero
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double cx = t[h][0] - st.u[0], cy = t[h][1] - st.u[1], cz = t[h][2] - st.u[2];
            const double c2 = cx * cx + cy * cy + cz * cz;
            const double phi[5] = {1.0, cx, cy, cz, c2};
#pragma unroll
            for (int sh = 0; sh < NSH; ++sh) {
                const double E = t[h][3] * exp_core(fmax(-c2 * iT[sh], -745.0));
                const double sE = E * (1.0 + (qp[sh][0] * cx + qp[sh][1] * cy + qp[sh][2] * cz) * (c2 * iT[sh] - 2.5));
                int k = sh * NS;
#pragma unroll
                for (int i = 0; i < 5; ++i) {
                    const double ei = phi[i] * E;
#pragma unroll
                    for (int j = i; j < 5; ++j) acc[k++] += ei * phi[j];
                }
#pragma unroll
                for (int i = 0; i < 5; ++i) acc[k++] += phi[i] * sE;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NA; ++k) part[k][lane] = acc[k];
    __syncthreads();
    if (lane < NA) {
        double s = 0.0;
        for (int j = 0; j < 64; ++j) s += part[lane][j];
        d.lsum[(size_t)cell * LSUM + lane] = s;
    }
}

__global__ __launch_bounds__(64) void k_params_list_finish(GSIS_SPAN_ARGS)
{
    int blk;
    const Case &C = case_of(span_cases, span_map, blk);
    const Geo &g = C.g;
    const Dev &d = C.d;
    const int cell = blk * blockDim.x + threadIdx.x;
    if (cell >= g.ncell || !d.cflag[cell]) return;   // a solid cell's parameters are zero already
    CellState st;
    cell_state(g, d, cell, st);
    const double *sums = d.lsum + (size_t)cell * LSUM;
    const int nsh = g.species != 0 ? 2 : 1;
    ShapeSums E[2];
    for (int sh = 0; sh < nsh; ++sh) {
        int k = sh * LSUM_SHAPE;
        for (int i = 0; i < 5; ++i)
            for (int j = i; j < 5; ++j) E[sh].G[i * 5 + j] = E[sh].G[j * 5 + i] = sums[k++];
        for (int i = 0; i < 5; ++i) E[sh].bS[i] = sums[k++];
    }
    cell_params(g, d, cell, st, E[0], E[nsh - 1]);
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
    if (t.vlist) {
        const dim3 grid(t.host[0].g.ncell);
        if (t.dia) hipLaunchKernelGGL(k_params_list_sums<2>, grid, dim3(64), 0, s, GSIS_SPAN(t.span(K_CELL1)));
        else hipLaunchKernelGGL(k_params_list_sums<1>, grid, dim3(64), 0, s, GSIS_SPAN(t.span(K_CELL1)));
        hipLaunchKernelGGL(k_params_list_finish, dim3(t.nblk[K_CELL64]), dim3(64), 0, s, GSIS_SPAN(t.span(K_CELL64)));
        return hipGetLastError();
    }
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

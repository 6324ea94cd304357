/*
 * gsis_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
 *
 * A plain, slow, FP64 CPU implementation of one GSIS iteration of the
 * discrete velocity method of arXiv 2310.18916 ("Efficient parallel solver
 * for rarefied gas flow using GSIS").  It exists only so that the GPU path
 * can be checked against something written straight from the equations.
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * load it.  It shares no code, header, table or constant with the HIP
 * library: everything below is written out again from the paper.
 *
 * Units (dimensionless): x in L, molecular velocity xi in v_m = sqrt(2 R T0),
 * rho in rho0, T in T0, time in L / v_m.  In these units R T -> T / 2, the
 * Maxwellian is rho (pi T)^{-3/2} exp(-|c|^2 / T), the collision rate is
 * 1/tau = delta rho T_t^{1-omega} with delta = sqrt(pi) / (2 Kn) (Sec. 2.1,
 * definition of Kn and the power-law viscosity), sigma is in p0 and q in
 * p0 v_m.
 *
 * What each function follows:
 *   moments            Eq. (getmoment), two-pass central sums, Neumaier.
 *   reference dists    Sec. 2.2, reference distributions g_0t, g_0r, g_1t,
 *                      g_1r and the q0/q1 mixing matrix; the Rykov mixture
 *                      g = (1 - 1/Z_r) g_t + g_r / Z_r of Sec. 3.2.
 *   conservative fix   not in the paper (it cites a conservative DVM): the
 *                      reference distribution is corrected by M (lambda.phi),
 *                      phi = (1, xi, |xi|^2), so that its discrete moments
 *                      equal their continuous values exactly.
 *   sweep              Sec. 3.2, backward-Euler kinetic update in delta form
 *                      with first-order upwind fluxes on both sides, solved
 *                      exactly by visiting cells in upwind order; or (order
 *                      2) the same first-order left-hand side with the
 *                      right-hand side's interface values reconstructed to
 *                      second order (least-squares gradient, Venkatakrishnan
 *                      limiter), solved for the increment.  On an
 *                      unstructured mesh (cells with volumes, faces with
 *                      areas and normals) the first-order update of the
 *                      same equation, cells visited in a topological order
 *                      of each node's upwind graph.
 *   boundary           diffuse wall (discrete half-range zero mass flux, wall
 *                      density lagged to f^n) and Maxwellian inflow.
 *   gsis_correct       Sec. 3.3, GSIS-II macroscopic equations with the
 *                      high-order terms of Eq. (full_constitutive), Rusanov
 *                      convective flux, the diagonal of Eq. (res_macro) in a
 *                      point-Jacobi iteration, then Eq. (updatef); on an
 *                      unstructured mesh the same solve over faces of any
 *                      normal (least-squares cell gradients).
 *   residual           Eq. (convergence_critertion), Sec. 5.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#include <omp.h>

#define ORC_NBC 7
#define ORC_WALL 0
#define ORC_INFLOW 1

typedef struct {
    int nx, ny, nz;
    double lx, ly, lz;
    int nv[3];
    double vmin[3], vmax[3];
    int species;            /* 0 monatomic Shakhov, 1 diatomic Rykov (two VDFs) */
    double Kn, omega;
    double dr, Zr, A[4];    /* diatomic only: internal DOF, collision number, A_tt A_tr A_rt A_rr */
    double inv_dt;          /* 1/Delta t of the kinetic update; 0 = source iteration */
    int conservative;       /* 1: moment-matched reference distribution */
    double macro_cfl;
    int bc_kind[ORC_NBC];   /* faces -x,+x,-y,+y,-z,+z of the box, then the solid surface */
    double bc_u[ORC_NBC][3];
    double bc_T[ORC_NBC];
    double bc_rho[ORC_NBC];
    /* optional per-axis node positions (strictly increasing, nv[a] of them);
     * NULL: nv[a] uniform nodes on [vmin, vmax].  Read once, at creation. */
    const double *nodes[3];
    /* spatial order of the explicit interface values of the kinetic update:
     * 1 first-order upwind, 2 second-order reconstruction (Sec. 3.2); and
     * the Venkatakrishnan constant K (eps^2 = (K h)^3 times the square of the
     * local largest |f|; K < 0: no limiter) */
    int order;
    double limiter_k;
    /* optional general velocity set (Sec. 3.1: a locally refined or
     * unstructured velocity mesh, each node standing for one velocity cell):
     * nlist > 0 nodes, node_list[4 k + 0..2] = xi of node k and
     * node_list[4 k + 3] = its weight, the volume of its cell.  Replaces the
     * tensor grid (nv, vmin, vmax, nodes are then ignored); read once, at
     * creation. */
    int nlist;
    const double *node_list;
    /* optional unstructured spatial mesh (Sec. 3.2: cells i of volume V_i,
     * interfaces ij of area S_ij and unit normal n pointing from i to j):
     * ucells > 0 cells replace the nx x ny x nz box (nx, ny, nz, lx, ly, lz and
     * the solid mask are then ignored); uface_cell[2 f] is the owner of face f,
     * uface_cell[2 f + 1] the neighbour cell or -1 - slot for a boundary face
     * of boundary slot 0..6; uface_geom[4 f] its area and [4 f + 1..3] its unit
     * normal out of the owner.  First order only; read once, at creation. */
    int ucells, ufaces;
    const double *uvol;
    const int *uface_cell;
    const double *uface_geom;
    /* cell centroids [ucells][3] and face centroids [ufaces][3] of the
     * unstructured mesh (the macroscopic correction's gradients and face
     * distances); NULL: kinetic passes only. */
    const double *ucenter, *ufcenter;
    /* macroscopic boundary flux of the correction (Sec. 3.3): 0 the cell's
     * Maxwellian (F_eq), 1 the Grad-13 reconstruction of Eq. (G13_VDF) from
     * the iterate and Eq. (full_constitutive) (F_G13); both enter as the
     * kinetic flux plus the change of the model flux from W^{n+1/2} to W^m. */
    int wall_flux;
} orc_cfg;

typedef struct {
    orc_cfg c;
    int ncell, nv;
    double h[3];
    double delta;
    unsigned char *solid;
    double *xi[3], *w1[3];
    double *f0, *f1;
    double *prev;           /* residual snapshot: rho, ux, uy, uz, Tt per cell */
    double *lastW;          /* W^{n+1} of the last macroscopic solve, [ncell][6] (NULL before one) */
    double *ntab;           /* [nv][4]: xi_x, xi_y, xi_z, weight of every node */
    double *mbw;            /* [ORC_NBC][nv] boundary Maxwellians M(1, u_b, T_b) at every node */
    double in_half[6][ORC_NBC]; /* sum_{xi_n < 0} w |xi_n| M(1, u_b, T_b) per face direction and slot */
    /* unstructured mesh (umesh = 1): copies of the cell volumes and faces, and
     * the faces of every cell, cf[cf_off[i] .. cf_off[i + 1]) = 2 f + side
     * (side 0: the cell owns face f, 1: it is the neighbour) */
    int umesh, nface;
    double *uvol, *ufg, *ucen, *ufcen;
    int *ufc, *cf_off, *cf;
    int status;
} orc_state;

/* ---------------------------------------------------------------- sums -- */
typedef struct { double s, c; } nsum;
static void nadd(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double nval(const nsum *a) { return a->s + a->c; }

/* --------------------------------------------------------------- setup -- */
static int cell_index(const orc_state *s, int i, int j, int k)
{
    return i + s->c.nx * (j + s->c.ny * k);
}

static void node_xi(const orc_state *s, int v, double xi[3], double *w)
{
    const double *t = s->ntab + (size_t)v * 4;
    xi[0] = t[0];
    xi[1] = t[1];
    xi[2] = t[2];
    *w = t[3];
}

/* Node v (x fastest) of the tensor grid: its velocity and its weight, the
 * product of the three 1-D weights; or node v of a general node list as
 * given.  Tabulated once (node_xi reads it). */
static void fill_node_table(orc_state *s, const double *list)
{
    if (list) {
        memcpy(s->ntab, list, sizeof(double) * (size_t)s->nv * 4);
        return;
    }
    for (int v = 0; v < s->nv; ++v) {
        int kx = v % s->c.nv[0];
        int ky = (v / s->c.nv[0]) % s->c.nv[1];
        int kz = v / (s->c.nv[0] * s->c.nv[1]);
        double *t = s->ntab + (size_t)v * 4;
        t[0] = s->xi[0][kx];
        t[1] = s->xi[1][ky];
        t[2] = s->xi[2][kz];
        t[3] = s->w1[0][kx] * s->w1[1][ky] * s->w1[2][kz];
    }
}

void orc_free(orc_state *s)
{
    if (!s) return;
    free(s->solid);
    for (int a = 0; a < 3; ++a) { free(s->xi[a]); free(s->w1[a]); }
    free(s->f0); free(s->f1); free(s->prev); free(s->lastW); free(s->mbw); free(s->ntab);
    free(s->uvol); free(s->ufg); free(s->ufc); free(s->cf_off); free(s->cf); free(s->ucen); free(s->ufcen);
    free(s);
}

static double maxwellian(double rho, const double u[3], double T, const double xi[3]);

static int check_mesh(const orc_cfg *cfg)
{
    if (cfg->ufaces < 1 || !cfg->uvol || !cfg->uface_cell || !cfg->uface_geom || cfg->order != 1) return 0;
    for (int i = 0; i < cfg->ucells; ++i)
        if (!(cfg->uvol[i] > 0) || !isfinite(cfg->uvol[i])) return 0;
    for (int f = 0; f < cfg->ufaces; ++f) {
        int o = cfg->uface_cell[2 * f], n = cfg->uface_cell[2 * f + 1];
        const double *g = cfg->uface_geom + (size_t)f * 4;
        if (o < 0 || o >= cfg->ucells || n >= cfg->ucells || n == o || n < -ORC_NBC) return 0;
        if (!(g[0] >= 0) || !isfinite(g[0]) || !isfinite(g[1]) || !isfinite(g[2]) || !isfinite(g[3])) return 0;
    }
    return 1;
}

static orc_state *create_state(const orc_cfg *cfg, const unsigned char *solid, int with_vdf)
{
    const int um = cfg->ucells > 0;
    if (um && !check_mesh(cfg)) return NULL;
    if (!um && (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1)) return NULL;
    if (cfg->order != 1 && cfg->order != 2) return NULL;
    if (cfg->wall_flux != 0 && cfg->wall_flux != 1) return NULL;
    if (!isfinite(cfg->limiter_k)) return NULL;
    const int list = cfg->nlist > 0;
    if (cfg->nlist < 0 || (list && !cfg->node_list)) return NULL;
    for (int k = 0; k < cfg->nlist; ++k) {
        const double *t = cfg->node_list + (size_t)k * 4;
        if (!isfinite(t[0]) || !isfinite(t[1]) || !isfinite(t[2]) || !(t[3] > 0) || !isfinite(t[3])) return NULL;
    }
    for (int a = 0; a < 3 && !list; ++a) {
        if (cfg->nv[a] < 2) return NULL;
        if (cfg->nodes[a]) {
            for (int k = 0; k < cfg->nv[a]; ++k)
                if (!isfinite(cfg->nodes[a][k]) || (k > 0 && !(cfg->nodes[a][k] > cfg->nodes[a][k - 1]))) return NULL;
        } else if (!(cfg->vmax[a] > cfg->vmin[a])) {
            return NULL;
        }
    }
    orc_state *s = calloc(1, sizeof(*s));
    s->c = *cfg;
    s->ncell = um ? cfg->ucells : cfg->nx * cfg->ny * cfg->nz;
    s->nv = list ? cfg->nlist : cfg->nv[0] * cfg->nv[1] * cfg->nv[2];
    s->h[0] = cfg->lx / cfg->nx;
    s->h[1] = cfg->ly / cfg->ny;
    s->h[2] = cfg->lz / cfg->nz;
    s->delta = sqrt(M_PI) / (2.0 * cfg->Kn);
    s->solid = calloc((size_t)s->ncell, 1);
    if (solid && !um) memcpy(s->solid, solid, (size_t)s->ncell);
    if (um) {
        int nc = s->ncell, nf = cfg->ufaces;
        s->umesh = 1;
        s->nface = nf;
        s->uvol = malloc(sizeof(double) * nc);
        s->ufg = malloc(sizeof(double) * 4 * (size_t)nf);
        s->ufc = malloc(sizeof(int) * 2 * (size_t)nf);
        memcpy(s->uvol, cfg->uvol, sizeof(double) * nc);
        memcpy(s->ufg, cfg->uface_geom, sizeof(double) * 4 * (size_t)nf);
        memcpy(s->ufc, cfg->uface_cell, sizeof(int) * 2 * (size_t)nf);
        s->cf_off = calloc((size_t)nc + 1, sizeof(int));
        for (int f = 0; f < nf; ++f) {
            s->cf_off[s->ufc[2 * f] + 1]++;
            if (s->ufc[2 * f + 1] >= 0) s->cf_off[s->ufc[2 * f + 1] + 1]++;
        }
        for (int i = 0; i < nc; ++i) s->cf_off[i + 1] += s->cf_off[i];
        s->cf = malloc(sizeof(int) * (size_t)s->cf_off[nc]);
        int *at = malloc(sizeof(int) * nc);
        memcpy(at, s->cf_off, sizeof(int) * nc);
        for (int f = 0; f < nf; ++f) {
            s->cf[at[s->ufc[2 * f]]++] = 2 * f;
            if (s->ufc[2 * f + 1] >= 0) s->cf[at[s->ufc[2 * f + 1]]++] = 2 * f + 1;
        }
        free(at);
        if (cfg->ucenter && cfg->ufcenter) {
            s->ucen = malloc(sizeof(double) * 3 * (size_t)nc);
            s->ufcen = malloc(sizeof(double) * 3 * (size_t)nf);
            memcpy(s->ucen, cfg->ucenter, sizeof(double) * 3 * (size_t)nc);
            memcpy(s->ufcen, cfg->ufcenter, sizeof(double) * 3 * (size_t)nf);
        }
        s->c.uvol = NULL; s->c.uface_cell = NULL; s->c.uface_geom = NULL;   /* copied */
        s->c.ucenter = NULL; s->c.ufcenter = NULL;
    }
    for (int a = 0; a < 3 && !list; ++a) {
        int n = cfg->nv[a];
        double d = (cfg->vmax[a] - cfg->vmin[a]) / (n - 1);
        s->xi[a] = malloc(sizeof(double) * n);
        s->w1[a] = malloc(sizeof(double) * n);
        if (cfg->nodes[a]) {
            /* trapezoid rule on the given nodes: half of each neighbouring gap */
            const double *x = cfg->nodes[a];
            for (int k = 0; k < n; ++k) {
                s->xi[a][k] = x[k];
                s->w1[a][k] = 0.5 * ((k < n - 1 ? x[k + 1] : x[k]) - (k > 0 ? x[k - 1] : x[k]));
            }
        } else {
            for (int k = 0; k < n; ++k) {
                s->xi[a][k] = cfg->vmin[a] + k * d;
                s->w1[a][k] = (k == 0 || k == n - 1) ? 0.5 * d : d;   /* trapezoid */
            }
        }
        s->c.nodes[a] = NULL;   /* copied: the caller's array is not kept */
    }
    s->prev = calloc((size_t)s->ncell * 5, sizeof(double));
    s->ntab = malloc(sizeof(double) * (size_t)s->nv * 4);
    fill_node_table(s, list ? cfg->node_list : NULL);
    for (int a = 0; a < 3; ++a) s->c.nodes[a] = NULL;
    s->c.node_list = NULL;   /* copied: the caller's array is not kept */
    /* the boundary Maxwellians do not change: tabulated once, with the incoming
     * half-range mass flux of each (face direction, slot) */
    s->mbw = malloc(sizeof(double) * (size_t)ORC_NBC * s->nv);
    for (int b = 0; b < ORC_NBC; ++b)
        for (int v = 0; v < s->nv; ++v) {
            double xi[3], w;
            node_xi(s, v, xi, &w);
            s->mbw[(size_t)b * s->nv + v] = maxwellian(1.0, cfg->bc_u[b], cfg->bc_T[b], xi);
        }
    for (int d = 0; d < 6; ++d)
        for (int b = 0; b < ORC_NBC; ++b) {
            int a = d / 2;
            double sg = (d & 1) ? 1.0 : -1.0;
            nsum in = {0, 0};
            for (int v = 0; v < s->nv; ++v) {
                double xi[3], w;
                node_xi(s, v, xi, &w);
                double xn = sg * xi[a];
                if (xn < 0) nadd(&in, w * (-xn) * s->mbw[(size_t)b * s->nv + v]);
            }
            s->in_half[d][b] = nval(&in);
        }
    if (!with_vdf) return s;
    size_t np = (size_t)s->ncell * s->nv;
    s->f0 = calloc(np, sizeof(double));
    if (cfg->species == 1) s->f1 = calloc(np, sizeof(double));
    if (!s->f0 || (cfg->species == 1 && !s->f1)) { orc_free(s); return NULL; }
    return s;
}

orc_state *orc_create(const orc_cfg *cfg, const unsigned char *solid)
{
    return create_state(cfg, solid, 1);
}

int orc_ncell(const orc_state *s) { return s->ncell; }
int orc_nv(const orc_state *s) { return s->nv; }
int orc_status(const orc_state *s) { return s->status; }

/* Maxwellian rho (pi T)^{-3/2} exp(-|xi-u|^2/T) in the units above. */
static double maxwellian(double rho, const double u[3], double T, const double xi[3])
{
    double c2 = 0;
    for (int a = 0; a < 3; ++a) c2 += (xi[a] - u[a]) * (xi[a] - u[a]);
    return rho * pow(M_PI * T, -1.5) * exp(-c2 / T);
}

/* The same value with pre = pow(M_PI * T, -1.5) computed by the caller once
 * for many nodes (identical operations, so identical results). */
static double maxwellian_pre(double rho, double pre, const double u[3], double T, const double xi[3])
{
    double c2 = 0;
    for (int a = 0; a < 3; ++a) c2 += (xi[a] - u[a]) * (xi[a] - u[a]);
    return rho * pre * exp(-c2 / T);
}

/* ------------------------------------------------------------- moments -- */
typedef struct {
    double rho, u[3], Tt, sig[6], q[3];   /* sigma order xx yy zz xy xz yz */
    double Tr, qr[3], T;
} moms;

/* Eq. (getmoment), written in the units above:
 *   rho = sum w f0,  rho u = sum w xi f0,  (3/2) rho Tt = sum w |c|^2 f0,
 *   sigma = 2 sum w (c c - |c|^2 I / 3) f0,  q = sum w c |c|^2 f0,
 *   (dr/2) rho Tr = sum w f1,  qr = sum w c f1,  T = (3 Tt + dr Tr)/(3 + dr). */
static void cell_moments(const orc_state *s, int cell, moms *m)
{
    const double *f0 = s->f0 + (size_t)cell * s->nv;
    const double *f1 = s->f1 ? s->f1 + (size_t)cell * s->nv : NULL;
    nsum r = {0, 0}, mu[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int v = 0; v < s->nv; ++v) {
        double xi[3], w;
        node_xi(s, v, xi, &w);
        nadd(&r, w * f0[v]);
        for (int a = 0; a < 3; ++a) nadd(&mu[a], w * xi[a] * f0[v]);
    }
    m->rho = nval(&r);
    for (int a = 0; a < 3; ++a) m->u[a] = nval(&mu[a]) / m->rho;
    nsum cc[6] = {{0, 0}}, c3[3] = {{0, 0}}, e1 = {0, 0}, q1[3] = {{0, 0}};
    memset(cc, 0, sizeof cc); memset(c3, 0, sizeof c3); memset(q1, 0, sizeof q1);
    for (int v = 0; v < s->nv; ++v) {
        double xi[3], w, c[3];
        node_xi(s, v, xi, &w);
        for (int a = 0; a < 3; ++a) c[a] = xi[a] - m->u[a];
        double c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        double wf = w * f0[v];
        nadd(&cc[0], wf * c[0] * c[0]);
        nadd(&cc[1], wf * c[1] * c[1]);
        nadd(&cc[2], wf * c[2] * c[2]);
        nadd(&cc[3], wf * c[0] * c[1]);
        nadd(&cc[4], wf * c[0] * c[2]);
        nadd(&cc[5], wf * c[1] * c[2]);
        for (int a = 0; a < 3; ++a) nadd(&c3[a], wf * c[a] * c2);
        if (f1) {
            nadd(&e1, w * f1[v]);
            for (int a = 0; a < 3; ++a) nadd(&q1[a], w * c[a] * f1[v]);
        }
    }
    double S[6];
    for (int k = 0; k < 6; ++k) S[k] = nval(&cc[k]);
    double tr = S[0] + S[1] + S[2];
    m->Tt = (2.0 / 3.0) * tr / m->rho;
    for (int k = 0; k < 6; ++k) m->sig[k] = 2.0 * (S[k] - (k < 3 ? tr / 3.0 : 0.0));
    for (int a = 0; a < 3; ++a) m->q[a] = nval(&c3[a]);
    if (f1) {
        double dr = s->c.dr;
        m->Tr = 2.0 * nval(&e1) / (dr * m->rho);
        for (int a = 0; a < 3; ++a) m->qr[a] = nval(&q1[a]);
        m->T = (3.0 * m->Tt + dr * m->Tr) / (3.0 + dr);
    } else {
        m->Tr = m->Tt;
        m->qr[0] = m->qr[1] = m->qr[2] = 0.0;
        m->T = m->Tt;
    }
}

/* ---------------------------------------------- reference distribution -- */
/* Shakhov form of Sec. 2.2 (the bracket with 2/15 fixes Pr = 2/3):
 *   S = M(rho,u,T) [1 + (4/15) (q.c) / (rho T^2) (|c|^2/T - 5/2)]. */
static double shakhov(double rho, const double u[3], double T, const double q[3], const double xi[3])
{
    double c[3], c2 = 0, qc = 0;
    for (int a = 0; a < 3; ++a) { c[a] = xi[a] - u[a]; c2 += c[a] * c[a]; qc += q[a] * c[a]; }
    double M = rho * pow(M_PI * T, -1.5) * exp(-c2 / T);
    return M * (1.0 + (4.0 / 15.0) * qc / (rho * T * T) * (c2 / T - 2.5));
}

/* Extra term of g_1t / g_1r: 2 (pi T)^{-3/2} (qr.c / T) exp(-|c|^2/T). */
static double rot_flux_term(const double u[3], double T, const double qr[3], const double xi[3])
{
    double c2 = 0, qc = 0;
    for (int a = 0; a < 3; ++a) { double c = xi[a] - u[a]; c2 += c * c; qc += qr[a] * c; }
    return 2.0 * pow(M_PI * T, -1.5) * (qc / T) * exp(-c2 / T);
}

typedef struct {
    moms m;
    double q0[3], q1[3];
    double lam_t[5], lam_r[5], nu_t, nu_r;
    double invtau;
} cellpar;

/* The four uncorrected reference components of Sec. 2.2 at one node. */
static void ref_components(const orc_cfg *c, const cellpar *p, const double xi[3], double out[4])
{
    const moms *m = &p->m;
    double S0t = shakhov(m->rho, m->u, m->Tt, m->q, xi);
    out[0] = S0t;
    if (c->species == 0) { out[1] = out[2] = out[3] = 0.0; return; }
    double S0r = shakhov(m->rho, m->u, m->T, p->q0, xi);
    out[1] = S0r;
    out[2] = 0.5 * c->dr * m->Tr * S0t + rot_flux_term(m->u, m->Tt, m->qr, xi);
    out[3] = 0.5 * c->dr * m->T * S0r + rot_flux_term(m->u, m->T, p->q1, xi);
}

static void phi5(const double xi[3], double phi[5])
{
    phi[0] = 1.0; phi[1] = xi[0]; phi[2] = xi[1]; phi[3] = xi[2];
    phi[4] = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
}

/* Dense solve with partial pivoting; n <= 5.  A pivot below 1e-12 of the
 * largest entry of A counts as zero: the system is singular (returns -1). */
static int solve_dense(int n, double *A, double *b)
{
    double amax = 0.0;
    for (int i = 0; i < n * n; ++i) amax = fmax(amax, fabs(A[i]));
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i) if (fabs(A[i * n + k]) > fabs(A[piv * n + k])) piv = i;
        if (!(fabs(A[piv * n + k]) > 1e-12 * amax)) return -1;
        if (piv != k) {
            for (int j = 0; j < n; ++j) { double t = A[k * n + j]; A[k * n + j] = A[piv * n + j]; A[piv * n + j] = t; }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            double f = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            b[i] -= f * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double t = b[k];
        for (int j = k + 1; j < n; ++j) t -= A[k * n + j] * b[j];
        b[k] = t / A[k * n + k];
    }
    return 0;
}

/* Per-cell parameters: moments, collision rate, q0/q1 mixing and the
 * conservative correction.  The correction of a component X with
 * Maxwellian shape M_X solves  [sum w phi phi^T M_X] lambda = target - sum w phi S_X,
 * target = (rho, rho u, rho |u|^2 + (3/2) rho T_X), brute force over every node. */
static void params_from_moments(const orc_state *s, const moms *mom, cellpar *p)
{
    const orc_cfg *c = &s->c;
    memset(p, 0, sizeof(*p));
    p->m = *mom;
    const moms *m = &p->m;
    p->invtau = s->delta * m->rho * pow(m->Tt, 1.0 - c->omega);
    if (c->species == 1) {
        double Z = c->Zr;
        double Att = c->A[0], Atr = c->A[1], Art = c->A[2], Arr = c->A[3];
        for (int a = 0; a < 3; ++a) {
            p->q0[a] = ((2.0 - 3.0 * Att) * Z + 1.0) * m->q[a] + (-3.0 * Atr * Z) * m->qr[a];
            p->q1[a] = (-Art * Z) * m->q[a] + (-Arr * Z + 1.0) * m->qr[a];
        }
    }
    if (!c->conservative) return;
    int ncomp = c->species == 1 ? 2 : 1;
    for (int X = 0; X < ncomp; ++X) {
        double TX = X == 0 ? m->Tt : m->T;
        double G[25] = {0}, b[5] = {0};
        nsum Gs[25], bs[5];
        memset(Gs, 0, sizeof Gs); memset(bs, 0, sizeof bs);
        for (int v = 0; v < s->nv; ++v) {
            double xi[3], w, ph[5], comp[4];
            node_xi(s, v, xi, &w);
            phi5(xi, ph);
            double MX = maxwellian(m->rho, m->u, TX, xi);
            ref_components(c, p, xi, comp);
            double SX = comp[X];
            for (int i = 0; i < 5; ++i) {
                nadd(&bs[i], w * ph[i] * SX);
                for (int j = 0; j < 5; ++j) nadd(&Gs[i * 5 + j], w * ph[i] * ph[j] * MX);
            }
        }
        double u2 = m->u[0] * m->u[0] + m->u[1] * m->u[1] + m->u[2] * m->u[2];
        double target[5] = {m->rho, m->rho * m->u[0], m->rho * m->u[1], m->rho * m->u[2],
                            m->rho * u2 + 1.5 * m->rho * TX};
        for (int i = 0; i < 5; ++i) {
            b[i] = target[i] - nval(&bs[i]);
            for (int j = 0; j < 5; ++j) G[i * 5 + j] = nval(&Gs[i * 5 + j]);
        }
        /* A grid on which (1, xi, |xi|^2) are linearly dependent (e.g. two
         * nodes +-a on every axis: |xi|^2 is constant) cannot match mass and
         * energy separately: the correction is then not applied. */
        if (solve_dense(5, G, b) != 0) memset(b, 0, sizeof b);
        memcpy(X == 0 ? p->lam_t : p->lam_r, b, sizeof b);
    }
    if (c->species == 1) {
        /* g_1t and g_1r: one constraint each, sum w g_1X = (dr/2) rho T_X'. */
        nsum s1t = {0, 0}, s1r = {0, 0}, mt = {0, 0}, mr = {0, 0};
        for (int v = 0; v < s->nv; ++v) {
            double xi[3], w, comp[4];
            node_xi(s, v, xi, &w);
            ref_components(c, p, xi, comp);
            nadd(&s1t, w * comp[2]);
            nadd(&s1r, w * comp[3]);
            nadd(&mt, w * maxwellian(m->rho, m->u, m->Tt, xi));
            nadd(&mr, w * maxwellian(m->rho, m->u, m->T, xi));
        }
        p->nu_t = (0.5 * c->dr * m->rho * m->Tr - nval(&s1t)) / nval(&mt);
        p->nu_r = (0.5 * c->dr * m->rho * m->T - nval(&s1r)) / nval(&mr);
    }
}

static void cell_params(const orc_state *s, int cell, cellpar *p)
{
    moms m;
    cell_moments(s, cell, &m);
    params_from_moments(s, &m, p);
}

/* The relaxation targets g0, g1 at one node (corrected components mixed
 * as g = (1 - 1/Z) g_t + g_r / Z; monatomic: g0 = corrected S). */
static void ref_dist(const orc_cfg *c, const cellpar *p, const double xi[3], double *g0, double *g1)
{
    const moms *m = &p->m;
    double comp[4], ph[5];
    ref_components(c, p, xi, comp);
    phi5(xi, ph);
    double Mt = maxwellian(m->rho, m->u, m->Tt, xi);
    double lt = 0;
    for (int i = 0; i < 5; ++i) lt += p->lam_t[i] * ph[i];
    double g0t = comp[0] + Mt * lt;
    if (c->species == 0) { *g0 = g0t; *g1 = 0.0; return; }
    double Mr = maxwellian(m->rho, m->u, m->T, xi);
    double lr = 0;
    for (int i = 0; i < 5; ++i) lr += p->lam_r[i] * ph[i];
    double g0r = comp[1] + Mr * lr;
    double g1t = comp[2] + p->nu_t * Mt;
    double g1r = comp[3] + p->nu_r * Mr;
    double iz = 1.0 / c->Zr;
    *g0 = (1.0 - iz) * g0t + iz * g0r;
    *g1 = (1.0 - iz) * g1t + iz * g1r;
}

/* ------------------------------------------------------------ boundary -- */
/* Neighbour of a fluid cell across face d (0:-x 1:+x 2:-y 3:+y 4:-z 5:+z):
 * returns the fluid cell index, or -1 - bc (bc = d for the box faces, 6 for
 * the solid surface). */
static int neighbour(const orc_state *s, int cell, int d)
{
    int nx = s->c.nx, ny = s->c.ny, nz = s->c.nz;
    int i = cell % nx, j = (cell / nx) % ny, k = cell / (nx * ny);
    int a = d / 2, sg = (d & 1) ? 1 : -1;
    int ii = i + (a == 0 ? sg : 0), jj = j + (a == 1 ? sg : 0), kk = k + (a == 2 ? sg : 0);
    if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) return -1 - d;
    int nb = cell_index(s, ii, jj, kk);
    if (s->solid[nb]) return -1 - 6;
    return nb;
}

/* Density scale of the incoming half of a boundary face.  Diffuse wall:
 * rho_w = sum_{xi.n>0} w xi.n f0 / sum_{xi.n<0} w |xi.n| M(1,u_w,T_w), so the
 * discrete mass flux through the wall is zero; inflow: the fixed density. */
static double face_scale(const orc_state *s, int cell, int d, int bc)
{
    const orc_cfg *c = &s->c;
    if (c->bc_kind[bc] == ORC_INFLOW) return c->bc_rho[bc];
    int a = d / 2;
    double sg = (d & 1) ? 1.0 : -1.0;
    const double *f0 = s->f0 + (size_t)cell * s->nv;
    nsum out = {0, 0}, in = {0, 0};
    for (int v = 0; v < s->nv; ++v) {
        double xi[3], w;
        node_xi(s, v, xi, &w);
        double xn = sg * xi[a];
        if (xn > 0) nadd(&out, w * xn * f0[v]);
        else if (xn < 0) nadd(&in, w * (-xn) * maxwellian(1.0, c->bc_u[bc], c->bc_T[bc], xi));
    }
    return nval(&out) / nval(&in);
}

/* Incoming boundary values f0_b, f1_b (f1 = (dr/2) T_b f0 for the equilibrium). */
static void boundary_value(const orc_cfg *c, int bc, double scale, const double xi[3], double *b0, double *b1)
{
    *b0 = scale * maxwellian(1.0, c->bc_u[bc], c->bc_T[bc], xi);
    *b1 = 0.5 * c->dr * c->bc_T[bc] * (*b0);
}

void orc_init_maxwellian(orc_state *s, double rho, const double u[3], double T, double Tr);

/* --------------------------------------------------------------- sweep -- */
/* The kinetic update of one velocity node v over all cells: Sec. 3.2,
 * backward Euler in pseudo time with first-order upwind fluxes.  With
 * a_a = |xi_a| / h_a, for fluid cell i
 *   f_i^{n+1/2} = [f_i^n / dt + g_i / tau_i + sum_a a_a F_a] / (1/dt + 1/tau_i + sum_a a_a),
 * F_a = f^{n+1/2} of the upwind cell, or the boundary value of the shared face.
 * Cells are visited in the upwind lexicographic order of the node's octant,
 * which solves the lower-triangular system exactly.  col0 (col1) holds the
 * node's values of every cell: f^n on entry, f^{n+1/2} on return. */
static void sweep_node(const orc_state *s, int v, const cellpar *P, const double *scale, const int *nb,
                       double *col0, double *col1)
{
    const orc_cfg *c = &s->c;
    int dia = c->species == 1;
    int nx = c->nx, ny = c->ny, nz = c->nz;
    double xi[3], w;
    node_xi(s, v, xi, &w);
    int sg[3];
    double aa[3];
    for (int a = 0; a < 3; ++a) { sg[a] = xi[a] >= 0 ? 1 : -1; aa[a] = fabs(xi[a]) / s->h[a]; }
    for (int kk = 0; kk < nz; ++kk) {
        int k = sg[2] > 0 ? kk : nz - 1 - kk;
        for (int jj = 0; jj < ny; ++jj) {
            int j = sg[1] > 0 ? jj : ny - 1 - jj;
            for (int ii = 0; ii < nx; ++ii) {
                int i = sg[0] > 0 ? ii : nx - 1 - ii;
                int cell = cell_index(s, i, j, k);
                if (s->solid[cell]) continue;
                double g0, g1;
                ref_dist(c, &P[cell], xi, &g0, &g1);
                double it = P[cell].invtau;
                double num0 = c->inv_dt * col0[cell] + it * g0;
                double num1 = dia ? c->inv_dt * col1[cell] + it * g1 : 0.0;
                double den = c->inv_dt + it;
                for (int a = 0; a < 3; ++a) {
                    if (aa[a] == 0.0) continue;
                    int d = 2 * a + (sg[a] > 0 ? 0 : 1);   /* upwind face */
                    int n = nb[cell * 6 + d];
                    double F0, F1;
                    if (n >= 0) {
                        F0 = col0[n];
                        F1 = dia ? col1[n] : 0.0;
                    } else {
                        boundary_value(c, -1 - n, scale[cell * 6 + d], xi, &F0, &F1);
                    }
                    num0 += aa[a] * F0;
                    num1 += aa[a] * F1;
                    den += aa[a];
                }
                col0[cell] = num0 / den;
                if (dia) col1[cell] = num1 / den;
            }
        }
    }
}

/* ------------------------------------------------- unstructured sweep -- */
/* Face entry e = 2 f + side of cell i: the unit normal out of i, S_f / V_i and
 * what lies on the other side (a cell, or -1 - slot for a boundary face). */
static void uface_of(const orc_state *s, int i, int e, double n[3], double *sv, int *other)
{
    int f = e >> 1, side = e & 1;
    const double *g = s->ufg + (size_t)f * 4;
    double sg = side ? -1.0 : 1.0;
    n[0] = sg * g[1];
    n[1] = sg * g[2];
    n[2] = sg * g[3];
    *sv = g[0] / s->uvol[i];
    *other = side ? s->ufc[2 * f] : s->ufc[2 * f + 1];
}

/* Density scale of the incoming half of boundary face f (unit normal n out
 * of its cell) from the f0 row of its cell: diffuse wall rho_w = sum_{xi.n>0} w xi.n f0 /
 * sum_{xi.n<0} w |xi.n| M(1,u_w,T_w) (zero discrete mass flux through the
 * wall), inflow the fixed density. */
static double uface_scale_row(const orc_state *s, int f, const double *f0)
{
    const orc_cfg *c = &s->c;
    int bc = -1 - s->ufc[2 * f + 1];
    if (c->bc_kind[bc] == ORC_INFLOW) return c->bc_rho[bc];
    const double *g = s->ufg + (size_t)f * 4;
    nsum out = {0, 0}, in = {0, 0};
    for (int v = 0; v < s->nv; ++v) {
        double xi[3], w;
        node_xi(s, v, xi, &w);
        double xn = xi[0] * g[1] + xi[1] * g[2] + xi[2] * g[3];
        if (xn > 0) nadd(&out, w * xn * f0[v]);
        else if (xn < 0) nadd(&in, w * (-xn) * s->mbw[(size_t)bc * s->nv + v]);
    }
    return nval(&out) / nval(&in);
}

static double uface_scale(const orc_state *s, int f)
{
    return uface_scale_row(s, f, s->f0 + (size_t)s->ufc[2 * f] * s->nv);
}

/* The kinetic update of node v on an unstructured mesh: Eq.
 * (delta_equations) with first-order upwind interface values on both sides.
 * With a_ij = (xi . n_ij) S_ij / V_i over the faces of cell i,
 *   f_i^{n+1/2} = [f_i^n / dt + g_i / tau_i + sum_{a_ij < 0} |a_ij| F_ij]
 *                 / (1/dt + 1/tau_i + sum_{a_ij > 0} a_ij),
 * F_ij the new value of neighbour j, or the boundary value of the face.  The
 * cells are visited in a topological order of the node's upwind graph (a
 * face carries the node from the cell it leaves into the cell it enters):
 * first the cells no face enters, then every cell once all cells upwind of it
 * are done (Kahn's algorithm), which solves the lower-triangular system
 * exactly.  A cycle in the graph -- a mesh that no sweep can order for this
 * node -- leaves cells unvisited and sets status -7. */
static void usweep_node(orc_state *s, int v, const cellpar *P, const double *bscale, double *col0, double *col1,
                        int *indeg, int *queue)
{
    const orc_cfg *c = &s->c;
    int dia = c->species == 1, nc = s->ncell;
    double xi[3], w;
    node_xi(s, v, xi, &w);
    for (int i = 0; i < nc; ++i) indeg[i] = 0;
    for (int f = 0; f < s->nface; ++f) {
        int o = s->ufc[2 * f], nb = s->ufc[2 * f + 1];
        if (nb < 0) continue;
        const double *g = s->ufg + (size_t)f * 4;
        double xn = xi[0] * g[1] + xi[1] * g[2] + xi[2] * g[3];
        if (xn > 0) indeg[nb]++;
        else if (xn < 0) indeg[o]++;
    }
    int head = 0, tail = 0;
    for (int i = 0; i < nc; ++i)
        if (indeg[i] == 0) queue[tail++] = i;
    while (head < tail) {
        int i = queue[head++];
        double g0, g1;
        ref_dist(c, &P[i], xi, &g0, &g1);
        double it = P[i].invtau;
        double num0 = c->inv_dt * col0[i] + it * g0;
        double num1 = dia ? c->inv_dt * col1[i] + it * g1 : 0.0;
        double den = c->inv_dt + it;
        for (int e = s->cf_off[i]; e < s->cf_off[i + 1]; ++e) {
            double n[3], sv;
            int other;
            uface_of(s, i, s->cf[e], n, &sv, &other);
            double a = (xi[0] * n[0] + xi[1] * n[1] + xi[2] * n[2]) * sv;
            if (a > 0) {
                den += a;
            } else if (a < 0) {
                double F0, F1;
                if (other >= 0) {
                    F0 = col0[other];
                    F1 = dia ? col1[other] : 0.0;
                } else {
                    boundary_value(c, -1 - other, bscale[s->cf[e] >> 1], xi, &F0, &F1);
                }
                num0 += -a * F0;
                num1 += -a * F1;
            }
        }
        col0[i] = num0 / den;
        if (dia) col1[i] = num1 / den;
        for (int e = s->cf_off[i]; e < s->cf_off[i + 1]; ++e) {
            double n[3], sv;
            int other;
            uface_of(s, i, s->cf[e], n, &sv, &other);
            if (other >= 0 && xi[0] * n[0] + xi[1] * n[1] + xi[2] * n[2] > 0 && --indeg[other] == 0)
                queue[tail++] = other;
        }
    }
    if (tail < nc) s->status = -7;
}

/* One kinetic pass on an unstructured mesh: per-cell parameters and boundary
 * densities from f^n, then every node swept on its own. */
static int one_pass_umesh(orc_state *s)
{
    const orc_cfg *c = &s->c;
    int ncell = s->ncell, nv = s->nv, dia = c->species == 1;
    cellpar *P = malloc(sizeof(cellpar) * (size_t)ncell);
    double *bscale = calloc((size_t)s->nface, sizeof(double));
    #pragma omp parallel for schedule(dynamic, 16)
    for (int cell = 0; cell < ncell; ++cell) cell_params(s, cell, &P[cell]);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int f = 0; f < s->nface; ++f)
        if (s->ufc[2 * f + 1] < 0) bscale[f] = uface_scale(s, f);
    for (int cell = 0; cell < ncell; ++cell)
        if (!isfinite(P[cell].invtau) || !(P[cell].m.rho > 0) || !(P[cell].m.Tt > 0)) s->status = -5;
    #pragma omp parallel
    {
        double *col0 = malloc(sizeof(double) * (size_t)ncell);
        double *col1 = dia ? malloc(sizeof(double) * (size_t)ncell) : NULL;
        int *indeg = malloc(sizeof(int) * (size_t)ncell), *queue = malloc(sizeof(int) * (size_t)ncell);
        #pragma omp for schedule(dynamic, 1)
        for (int v = 0; v < nv; ++v) {
            for (int cell = 0; cell < ncell; ++cell) {
                col0[cell] = s->f0[(size_t)cell * nv + v];
                if (dia) col1[cell] = s->f1[(size_t)cell * nv + v];
            }
            usweep_node(s, v, P, bscale, col0, col1, indeg, queue);
            for (int cell = 0; cell < ncell; ++cell) {
                s->f0[(size_t)cell * nv + v] = col0[cell];
                if (dia) s->f1[(size_t)cell * nv + v] = col1[cell];
            }
        }
        free(col0); free(col1); free(indeg); free(queue);
    }
    free(P); free(bscale);
    return s->status;
}

/* ------------------------------------------------ second-order values -- */
/* Sec. 3.2: the interface values in the right-hand side of Eq.
 * (delta_equations) come from a second-order upwind reconstruction,
 * f_ij = f_up + phi_up grad f_up . (x_ij - x_up), with the gradient from a
 * least-squares fit and phi the Venkatakrishnan limiter; the increments on
 * the left-hand side stay first-order upwind.  What the paper leaves open is
 * read as follows:
 *  - only faces between two fluid cells are reconstructed.  A box face or a
 *    solid surface keeps its first-order values (the cell's own value going
 *    out, the boundary value coming in), so the zero-mass-flux wall density
 *    is computed exactly as in the first-order scheme;
 *  - the least-squares fit runs over the fluid face neighbours.  Their offsets
 *    are axis-aligned, so the normal matrix is diagonal and each component is
 *    a 1-D fit; an axis with no fluid neighbour gets a zero component (the
 *    minimum-norm solution);
 *  - Venkatakrishnan's limiter: phi_i is the minimum over the reconstructed
 *    faces of psi(D, d2), with d2 = grad f_i . (x_ij - x_i) and D the largest
 *    (d2 > 0) or smallest (d2 < 0) of f_j - f_i over the cell and its fluid
 *    neighbours, psi = (D^2 + e2 + 2 D d2) / (D^2 + 2 d2^2 + D d2 + e2) and
 *    psi = 1 for d2 = 0; e2 = (K h)^3 S^2 with h the cube root of the cell
 *    volume, K = limiter_k and S the largest |f| over the cell and its fluid
 *    neighbours (the threshold relative to the local size of f, which spans
 *    decades across velocity space); K < 0 leaves the reconstruction
 *    unlimited (phi = 1). */
static void lsq_gradient(const orc_state *s, const int *nb, const double *col, int cell, double g[3])
{
    double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, b[3] = {0, 0, 0};
    for (int d = 0; d < 6; ++d) {
        int n = nb[cell * 6 + d];
        if (n < 0) continue;
        double off[3] = {0, 0, 0};
        off[d / 2] = ((d & 1) ? 1.0 : -1.0) * s->h[d / 2];
        for (int p = 0; p < 3; ++p) {
            for (int q = 0; q < 3; ++q) A[p][q] += off[p] * off[q];
            b[p] += off[p] * (col[n] - col[cell]);
        }
    }
    for (int p = 0; p < 3; ++p) g[p] = A[p][p] > 0 ? b[p] / A[p][p] : 0.0;   /* A is diagonal */
}

static double venkatakrishnan(double D, double d2, double e2)
{
    if (d2 == 0.0) return 1.0;
    return (D * D + e2 + 2.0 * D * d2) / (D * D + 2.0 * d2 * d2 + D * d2 + e2);
}

/* offset of face d from the cell centre along its axis */
static double face_offset(const orc_state *s, int d)
{
    return ((d & 1) ? 0.5 : -0.5) * s->h[d / 2];
}

static double limiter(const orc_state *s, const int *nb, const double *col, int cell, const double g[3])
{
    double K = s->c.limiter_k;
    if (K < 0) return 1.0;
    double hc = cbrt(s->h[0] * s->h[1] * s->h[2]);
    double e2 = (K * hc) * (K * hc) * (K * hc);
    double fi = col[cell], fmax = fi, fmin = fi;
    for (int d = 0; d < 6; ++d) {
        int n = nb[cell * 6 + d];
        if (n < 0) continue;
        if (col[n] > fmax) fmax = col[n];
        if (col[n] < fmin) fmin = col[n];
    }
    double S = fabs(fmax) > fabs(fmin) ? fabs(fmax) : fabs(fmin);
    e2 *= S * S;
    double phi = 1.0;
    for (int d = 0; d < 6; ++d) {
        if (nb[cell * 6 + d] < 0) continue;
        double d2 = g[d / 2] * face_offset(s, d);
        double psi = venkatakrishnan(d2 > 0 ? fmax - fi : fmin - fi, d2, e2);
        if (psi < phi) phi = psi;
    }
    return phi;
}

/* Value of every fluid cell at each of its faces, fv[cell][6]: reconstructed
 * at faces shared with a fluid cell when order = 2, the cell value otherwise. */
static void face_values(const orc_state *s, const int *nb, const double *col, int order, double *fv)
{
    for (int cell = 0; cell < s->ncell; ++cell) {
        if (s->solid[cell]) continue;
        double g[3] = {0, 0, 0}, phi = 0.0;
        if (order == 2) {
            lsq_gradient(s, nb, col, cell, g);
            phi = limiter(s, nb, col, cell, g);
        }
        for (int d = 0; d < 6; ++d)
            fv[cell * 6 + d] = col[cell] + (order == 2 && nb[cell * 6 + d] >= 0
                                            ? phi * g[d / 2] * face_offset(s, d) : 0.0);
    }
}

/* (1/V) sum_j xi_n f_ij S_ij of every fluid cell for node xi: the upwind face
 * value (fv of the upwind cell, or the boundary value bv[cell][6] on a box or
 * solid face) times the normal velocity, over the six faces. */
static void flux_divergence(const orc_state *s, const int *nb, const double *fv, const double *bv,
                            const double xi[3], double *div)
{
    for (int cell = 0; cell < s->ncell; ++cell) {
        if (s->solid[cell]) continue;
        double sum = 0.0;
        for (int d = 0; d < 6; ++d) {
            int a = d / 2;
            double xn = ((d & 1) ? 1.0 : -1.0) * xi[a];   /* outward normal velocity */
            double v;
            if (xn > 0) v = fv[cell * 6 + d];                              /* leaving: this cell */
            else if (nb[cell * 6 + d] >= 0) v = fv[nb[cell * 6 + d] * 6 + (d ^ 1)];   /* entering: neighbour */
            else v = bv[cell * 6 + d];                                     /* entering: boundary */
            sum += xn * v / s->h[a];
        }
        div[cell] = sum;
    }
}

/* The kinetic update of one node with the second-order right-hand side, in
 * the delta form of Sec. 3.2:
 *   (1/dt + 1/tau_i + sum_a a_a) Df_i - sum_{upwind fluid j} a_a Df_j = r_i,
 *   r_i = (g_i - f_i) / tau_i - (1/V) sum_j xi_n f_ij S_ij,
 * a_a = |xi_a| / h_a, with the increment of a boundary value zero (it is
 * lagged to f^n); solved in upwind order, then f^{n+1/2} = f^n + Df. */
static void sweep_node_second_order(const orc_state *s, int v, const cellpar *P, const double *scale, const int *nb,
                                    double *col0, double *col1)
{
    const orc_cfg *c = &s->c;
    int dia = c->species == 1, ncell = s->ncell;
    int nx = c->nx, ny = c->ny, nz = c->nz;
    double xi[3], w;
    node_xi(s, v, xi, &w);
    double *fv = malloc(sizeof(double) * (size_t)ncell * 6);
    double *bv = malloc(sizeof(double) * (size_t)ncell * 6);
    double *bv1 = malloc(sizeof(double) * (size_t)ncell * 6);
    double *r[2], *df[2];
    for (int q = 0; q < 2; ++q) { r[q] = calloc((size_t)ncell, sizeof(double)); df[q] = calloc((size_t)ncell, sizeof(double)); }
    for (int cell = 0; cell < ncell; ++cell) {
        if (s->solid[cell]) continue;
        for (int d = 0; d < 6; ++d) {
            int n = nb[cell * 6 + d];
            bv[cell * 6 + d] = bv1[cell * 6 + d] = 0.0;
            if (n < 0) boundary_value(c, -1 - n, scale[cell * 6 + d], xi, &bv[cell * 6 + d], &bv1[cell * 6 + d]);
        }
    }
    for (int q = 0; q < 1 + dia; ++q) {
        double *col = q ? col1 : col0;
        face_values(s, nb, col, 2, fv);
        flux_divergence(s, nb, fv, q ? bv1 : bv, xi, r[q]);
        for (int cell = 0; cell < ncell; ++cell) {
            if (s->solid[cell]) continue;
            double g0, g1;
            ref_dist(c, &P[cell], xi, &g0, &g1);
            r[q][cell] = ((q ? g1 : g0) - col[cell]) * P[cell].invtau - r[q][cell];
        }
    }
    int sg[3];
    double aa[3];
    for (int a = 0; a < 3; ++a) { sg[a] = xi[a] >= 0 ? 1 : -1; aa[a] = fabs(xi[a]) / s->h[a]; }
    for (int kk = 0; kk < nz; ++kk) {
        int k = sg[2] > 0 ? kk : nz - 1 - kk;
        for (int jj = 0; jj < ny; ++jj) {
            int j = sg[1] > 0 ? jj : ny - 1 - jj;
            for (int ii = 0; ii < nx; ++ii) {
                int i = sg[0] > 0 ? ii : nx - 1 - ii;
                int cell = cell_index(s, i, j, k);
                if (s->solid[cell]) continue;
                double den = c->inv_dt + P[cell].invtau;
                double num[2] = {r[0][cell], r[1][cell]};
                for (int a = 0; a < 3; ++a) {
                    if (aa[a] == 0.0) continue;
                    den += aa[a];
                    int n = nb[cell * 6 + 2 * a + (sg[a] > 0 ? 0 : 1)];
                    if (n < 0) continue;
                    num[0] += aa[a] * df[0][n];
                    num[1] += aa[a] * df[1][n];
                }
                df[0][cell] = num[0] / den;
                df[1][cell] = num[1] / den;
            }
        }
    }
    for (int cell = 0; cell < ncell; ++cell) {
        if (s->solid[cell]) continue;
        col0[cell] += df[0][cell];
        if (dia) col1[cell] += df[1][cell];
    }
    free(fv); free(bv); free(bv1);
    for (int q = 0; q < 2; ++q) { free(r[q]); free(df[q]); }
}

/* One kinetic pass: per-cell parameters and boundary densities from f^n,
 * then every node swept independently (the wall density is lagged), in place. */
static int one_pass(orc_state *s)
{
    if (s->umesh) return one_pass_umesh(s);
    const orc_cfg *c = &s->c;
    int ncell = s->ncell, nv = s->nv, dia = c->species == 1;
    cellpar *P = malloc(sizeof(cellpar) * (size_t)ncell);
    double *scale = malloc(sizeof(double) * (size_t)ncell * 6);
    int *nb = malloc(sizeof(int) * (size_t)ncell * 6);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int cell = 0; cell < ncell; ++cell) {
        if (s->solid[cell]) continue;
        cell_params(s, cell, &P[cell]);
        for (int d = 0; d < 6; ++d) {
            int n = neighbour(s, cell, d);
            nb[cell * 6 + d] = n;
            scale[cell * 6 + d] = n >= 0 ? 0.0 : face_scale(s, cell, d, -1 - n);
        }
    }
    for (int cell = 0; cell < ncell; ++cell) {
        if (s->solid[cell]) continue;
        if (!isfinite(P[cell].invtau) || !(P[cell].m.rho > 0) || !(P[cell].m.Tt > 0)) s->status = -5;
    }
    #pragma omp parallel
    {
        double *col0 = malloc(sizeof(double) * (size_t)ncell);
        double *col1 = dia ? malloc(sizeof(double) * (size_t)ncell) : NULL;
        #pragma omp for schedule(dynamic, 1)
        for (int v = 0; v < nv; ++v) {
            for (int cell = 0; cell < ncell; ++cell) {
                col0[cell] = s->f0[(size_t)cell * nv + v];
                if (dia) col1[cell] = s->f1[(size_t)cell * nv + v];
            }
            if (c->order == 2) sweep_node_second_order(s, v, P, scale, nb, col0, col1);
            else sweep_node(s, v, P, scale, nb, col0, col1);
            for (int cell = 0; cell < ncell; ++cell) {
                if (s->solid[cell]) continue;
                s->f0[(size_t)cell * nv + v] = col0[cell];
                if (dia) s->f1[(size_t)cell * nv + v] = col1[cell];
            }
        }
        free(col0);
        free(col1);
    }
    free(P); free(scale); free(nb);
    return s->status;
}

/* orc_first_pass_nodes on an unstructured mesh: every cell holds the same
 * f^n, so one cell's parameters serve all cells and each boundary face's wall
 * density comes from that one row; nodes swept as in one_pass_umesh. */
static int first_pass_nodes_umesh(const orc_cfg *cfg, double rho, const double u[3], double T, double Tr,
                                  const int *nodes, int nn, double *out0, double *out1)
{
    orc_cfg one = *cfg;
    one.ucells = one.ufaces = 0;
    one.uvol = NULL; one.uface_cell = NULL; one.uface_geom = NULL;
    one.nx = one.ny = one.nz = 1;
    one.lx = one.ly = one.lz = 1.0;
    orc_state *s1 = create_state(&one, NULL, 1);
    orc_state *s = create_state(cfg, NULL, 0);
    if (!s1 || !s) { orc_free(s1); orc_free(s); return -3; }
    orc_init_maxwellian(s1, rho, u, T, Tr);
    cellpar p1;
    cell_params(s1, 0, &p1);
    int status = (!isfinite(p1.invtau) || !(p1.m.rho > 0) || !(p1.m.Tt > 0)) ? -5 : 0;
    int ncell = s->ncell, dia = cfg->species == 1;
    cellpar *P = malloc(sizeof(cellpar) * (size_t)ncell);
    double *bscale = calloc((size_t)s->nface, sizeof(double));
    for (int cell = 0; cell < ncell; ++cell) P[cell] = p1;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int f = 0; f < s->nface; ++f)
        if (s->ufc[2 * f + 1] < 0) bscale[f] = uface_scale_row(s, f, s1->f0);
    #pragma omp parallel
    {
        int *indeg = malloc(sizeof(int) * (size_t)ncell), *queue = malloc(sizeof(int) * (size_t)ncell);
        #pragma omp for schedule(dynamic, 1)
        for (int k = 0; k < nn; ++k) {
            double *col0 = out0 + (size_t)k * ncell;
            double *col1 = dia ? out1 + (size_t)k * ncell : NULL;
            for (int cell = 0; cell < ncell; ++cell) {
                col0[cell] = s1->f0[nodes[k]];
                if (dia) col1[cell] = s1->f1[nodes[k]];
            }
            usweep_node(s, nodes[k], P, bscale, col0, col1, indeg, queue);
        }
        free(indeg); free(queue);
    }
    if (s->status) status = s->status;
    free(P); free(bscale);
    orc_free(s1);
    orc_free(s);
    return status;
}

/* The first pass from a uniform Maxwellian at selected nodes only, for
 * problems too large to hold the VDF: every fluid cell then has the same
 * f^n, so one cell's parameters and its wall densities (per face direction
 * and boundary slot) serve all cells, and the nodes are swept as in
 * one_pass.  out0[k][cell] (out1 for f1) = f^{n+1/2} at canonical node
 * nodes[k]; solid cells are 0.  Returns the status of the parameters. */
int orc_first_pass_nodes(const orc_cfg *cfg, const unsigned char *solid, double rho, const double u[3], double T,
                         double Tr, const int *nodes, int nn, double *out0, double *out1)
{
    if (cfg->ucells > 0) return first_pass_nodes_umesh(cfg, rho, u, T, Tr, nodes, nn, out0, out1);
    orc_cfg one = *cfg;
    one.nx = one.ny = one.nz = 1;
    orc_state *s1 = create_state(&one, NULL, 1);
    orc_state *s = create_state(cfg, solid, 0);
    if (!s1 || !s) { orc_free(s1); orc_free(s); return -3; }
    orc_init_maxwellian(s1, rho, u, T, Tr);
    cellpar p1;
    cell_params(s1, 0, &p1);
    int status = (!isfinite(p1.invtau) || !(p1.m.rho > 0) || !(p1.m.Tt > 0)) ? -5 : 0;
    double sc[6][ORC_NBC];
    for (int d = 0; d < 6; ++d)
        for (int b = 0; b < ORC_NBC; ++b) sc[d][b] = face_scale(s1, 0, d, b);
    int ncell = s->ncell, dia = cfg->species == 1;
    cellpar *P = malloc(sizeof(cellpar) * (size_t)ncell);
    double *scale = malloc(sizeof(double) * (size_t)ncell * 6);
    int *nb = malloc(sizeof(int) * (size_t)ncell * 6);
    for (int cell = 0; cell < ncell; ++cell) {
        P[cell] = p1;
        for (int d = 0; d < 6; ++d) {
            int n = neighbour(s, cell, d);
            nb[cell * 6 + d] = n;
            scale[cell * 6 + d] = n >= 0 ? 0.0 : sc[d][-1 - n];
        }
    }
    #pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < nn; ++k) {
        double *col0 = out0 + (size_t)k * ncell;
        double *col1 = dia ? out1 + (size_t)k * ncell : NULL;
        for (int cell = 0; cell < ncell; ++cell) {
            int fl = !s->solid[cell];
            col0[cell] = fl ? s1->f0[nodes[k]] : 0.0;
            if (dia) col1[cell] = fl ? s1->f1[nodes[k]] : 0.0;
        }
        sweep_node(s, nodes[k], P, scale, nb, col0, col1);
    }
    free(P); free(scale); free(nb);
    orc_free(s1);
    orc_free(s);
    return status;
}

int orc_step(orc_state *s, int npasses)
{
    for (int n = 0; n < npasses; ++n) one_pass(s);
    return s->status;
}

/* -------------------------------------------------------- state access -- */
static void snapshot(orc_state *s)
{
    for (int cell = 0; cell < s->ncell; ++cell) {
        double *pv = s->prev + (size_t)cell * 5;
        if (s->solid[cell]) { memset(pv, 0, 5 * sizeof(double)); continue; }
        moms m;
        cell_moments(s, cell, &m);
        pv[0] = m.rho; pv[1] = m.u[0]; pv[2] = m.u[1]; pv[3] = m.u[2]; pv[4] = m.Tt;
    }
}

void orc_init_maxwellian(orc_state *s, double rho, const double u[3], double T, double Tr)
{
    for (int cell = 0; cell < s->ncell; ++cell) {
        for (int v = 0; v < s->nv; ++v) {
            size_t at = (size_t)cell * s->nv + v;
            if (s->solid[cell]) { s->f0[at] = 0; if (s->f1) s->f1[at] = 0; continue; }
            double xi[3], w;
            node_xi(s, v, xi, &w);
            s->f0[at] = maxwellian(rho, u, T, xi);
            if (s->f1) s->f1[at] = 0.5 * s->c.dr * Tr * s->f0[at];
        }
    }
    s->status = 0;
    snapshot(s);
}

void orc_set_vdf(orc_state *s, const double *f0, const double *f1)
{
    size_t np = (size_t)s->ncell * s->nv;
    memcpy(s->f0, f0, np * sizeof(double));
    if (s->f1 && f1) memcpy(s->f1, f1, np * sizeof(double));
    s->status = 0;
    snapshot(s);
}

/* The VDF replaced without a new residual snapshot (the next residual
 * compares with the state before). */
void orc_replace_vdf(orc_state *s, const double *f0, const double *f1)
{
    size_t np = (size_t)s->ncell * s->nv;
    memcpy(s->f0, f0, np * sizeof(double));
    if (s->f1 && f1) memcpy(s->f1, f1, np * sizeof(double));
}

void orc_get_vdf(const orc_state *s, double *f0, double *f1)
{
    size_t np = (size_t)s->ncell * s->nv;
    memcpy(f0, s->f0, np * sizeof(double));
    if (s->f1 && f1) memcpy(f1, s->f1, np * sizeof(double));
}

/* out[ncell][14 or 18]: rho, ux, uy, uz, Tt, sxx, syy, szz, sxy, sxz, syz,
 * qx, qy, qz, [Tr, qrx, qry, qrz]; NaN in solid cells. */
void orc_moments(const orc_state *s, double *out)
{
    int nm = s->c.species == 1 ? 18 : 14;
    #pragma omp parallel for schedule(static)
    for (int cell = 0; cell < s->ncell; ++cell) {
        double *o = out + (size_t)cell * nm;
        if (s->solid[cell]) { for (int k = 0; k < nm; ++k) o[k] = NAN; continue; }
        moms m;
        cell_moments(s, cell, &m);
        o[0] = m.rho; o[1] = m.u[0]; o[2] = m.u[1]; o[3] = m.u[2]; o[4] = m.Tt;
        for (int k = 0; k < 6; ++k) o[5 + k] = m.sig[k];
        for (int a = 0; a < 3; ++a) o[11 + a] = m.q[a];
        if (nm == 18) { o[14] = m.Tr; for (int a = 0; a < 3; ++a) o[15 + a] = m.qr[a]; }
    }
}

/* Eq. (convergence_critertion), volume-weighted (uniform hex cells: weight 1); u is a vector.  A
 * denominator that is zero, or for u at most (1000 times the FP64 unit
 * roundoff)^2 times the sum of Tt^2 -- the velocity of a gas at rest is only
 * rounding noise -- reports the absolute change instead.  Compares with the
 * last snapshot and takes a new one. */
void orc_residual(orc_state *s, double eps[3])
{
    nsum num[3], den[3];
    memset(num, 0, sizeof num); memset(den, 0, sizeof den);
    for (int cell = 0; cell < s->ncell; ++cell) {
        if (s->solid[cell]) continue;
        moms m;
        cell_moments(s, cell, &m);
        const double *pv = s->prev + (size_t)cell * 5;
        double V = s->umesh ? s->uvol[cell] : 1.0;
        double dr = m.rho - pv[0], dT = m.Tt - pv[4];
        nadd(&num[0], V * dr * dr); nadd(&den[0], V * pv[0] * pv[0]);
        for (int a = 0; a < 3; ++a) {
            double du = m.u[a] - pv[1 + a];
            nadd(&num[1], V * du * du);
            nadd(&den[1], V * pv[1 + a] * pv[1 + a]);
        }
        nadd(&num[2], V * dT * dT); nadd(&den[2], V * pv[4] * pv[4]);
    }
    double ufloor = (1e3 * 2.220446049250313e-16) * (1e3 * 2.220446049250313e-16) * nval(&den[2]);
    for (int k = 0; k < 3; ++k) {
        double n = nval(&num[k]), d = nval(&den[k]);
        eps[k] = d > (k == 1 ? ufloor : 0.0) ? sqrt(n / d) : sqrt(n);
    }
    snapshot(s);
}

/* ---------------------------------------------------- pin/debug access -- */
/* Corrected relaxation targets g0, g1 of one cell at every node. */
void orc_ref_dist(const orc_state *s, int cell, double *g0, double *g1)
{
    cellpar p;
    cell_params(s, cell, &p);
    for (int v = 0; v < s->nv; ++v) {
        double xi[3], w, a, b;
        node_xi(s, v, xi, &w);
        ref_dist(&s->c, &p, xi, &a, &b);
        g0[v] = a;
        if (g1) g1[v] = b;
    }
}

/* Collision rate 1/tau of one cell from the current VDF. */
double orc_invtau(const orc_state *s, int cell)
{
    cellpar p;
    cell_params(s, cell, &p);
    return p.invtau;
}

/* Boundary values of face (cell, d) at every node (zero at nodes that leave
 * the cell through that face); returns the face's bc index, or -1 if the face
 * is interior. */
int orc_boundary_values(const orc_state *s, int cell, int d, double *b0, double *b1)
{
    if (s->umesh) return -2;
    int n = neighbour(s, cell, d);
    if (n >= 0) return -1;
    int bc = -1 - n;
    double sc = face_scale(s, cell, d, bc);
    int a = d / 2;
    double sg = (d & 1) ? 1.0 : -1.0;
    for (int v = 0; v < s->nv; ++v) {
        double xi[3], w, x0, x1;
        node_xi(s, v, xi, &w);
        boundary_value(&s->c, bc, sc, xi, &x0, &x1);
        int incoming = sg * xi[a] < 0;
        b0[v] = incoming ? x0 : 0.0;
        if (b1) b1[v] = incoming ? x1 : 0.0;
    }
    return bc;
}

/* The column of VDF `which` (0: f0, 1: f1) at canonical node v, the
 * neighbour table and the boundary values of every face, for the pins of
 * the second-order values. */
static void node_column(const orc_state *s, int v, int which, double *col, int *nb, double *bv)
{
    const double *f = which ? s->f1 : s->f0;
    double xi[3], w;
    node_xi(s, v, xi, &w);
    for (int cell = 0; cell < s->ncell; ++cell) {
        col[cell] = s->solid[cell] ? 0.0 : f[(size_t)cell * s->nv + v];
        for (int d = 0; d < 6; ++d) {
            int n = s->solid[cell] ? -1 : neighbour(s, cell, d);
            nb[cell * 6 + d] = n;
            double b0 = 0.0, b1 = 0.0;
            if (n < 0 && !s->solid[cell]) boundary_value(&s->c, -1 - n, face_scale(s, cell, d, -1 - n), xi, &b0, &b1);
            bv[cell * 6 + d] = which ? b1 : b0;
        }
    }
}

/* Face values fv[cell][6] of node v (order 1: the cell value; order 2: the
 * limited reconstruction on faces between fluid cells); NaN in solid cells. */
void orc_face_values(const orc_state *s, int v, int which, int order, double *fv)
{
    if (s->umesh) return;
    int ncell = s->ncell;
    double *col = malloc(sizeof(double) * ncell), *bv = malloc(sizeof(double) * ncell * 6);
    int *nb = malloc(sizeof(int) * ncell * 6);
    node_column(s, v, which, col, nb, bv);
    for (int k = 0; k < ncell * 6; ++k) fv[k] = NAN;
    face_values(s, nb, col, order, fv);
    free(col); free(bv); free(nb);
}

/* (1/V) sum_j xi_n f_ij S_ij of node v in every fluid cell with face values
 * of the given order and the current boundary values; NaN in solid cells. */
void orc_flux_divergence(const orc_state *s, int v, int which, int order, double *div)
{
    if (s->umesh) return;
    int ncell = s->ncell;
    double *col = malloc(sizeof(double) * ncell), *bv = malloc(sizeof(double) * ncell * 6);
    double *fv = malloc(sizeof(double) * ncell * 6);
    int *nb = malloc(sizeof(int) * ncell * 6);
    double xi[3], w;
    node_xi(s, v, xi, &w);
    node_column(s, v, which, col, nb, bv);
    for (int k = 0; k < ncell; ++k) div[k] = NAN;
    face_values(s, nb, col, order, fv);
    flux_divergence(s, nb, fv, bv, xi, div);
    free(col); free(bv); free(fv); free(nb);
}

/* The four uncorrected reference components (g0t, g0r, g1t, g1r) at n
 * arbitrary points, from given moments; for pins of Sec. 2.2. */
void orc_ref_components(const orc_cfg *c, double rho, const double u[3], double Tt, double Tr,
                        const double qt[3], const double qr[3], int n, const double *xi, double *out)
{
    cellpar p;
    memset(&p, 0, sizeof p);
    p.m.rho = rho;
    for (int a = 0; a < 3; ++a) { p.m.u[a] = u[a]; p.m.q[a] = qt[a]; p.m.qr[a] = qr ? qr[a] : 0.0; }
    p.m.Tt = Tt;
    p.m.Tr = c->species == 1 ? Tr : Tt;
    p.m.T = c->species == 1 ? (3.0 * Tt + c->dr * Tr) / (3.0 + c->dr) : Tt;
    if (c->species == 1) {
        double Z = c->Zr;
        for (int a = 0; a < 3; ++a) {
            p.q0[a] = ((2.0 - 3.0 * c->A[0]) * Z + 1.0) * p.m.q[a] + (-3.0 * c->A[1] * Z) * p.m.qr[a];
            p.q1[a] = (-c->A[2] * Z) * p.m.q[a] + (-c->A[3] * Z + 1.0) * p.m.qr[a];
        }
    }
    for (int i = 0; i < n; ++i) ref_components(c, &p, xi + 3 * i, out + 4 * i);
}

/* ------------------------------------------------------- gsis_correct -- */
/* GSIS-II (Sec. 3.3).  Unknowns per fluid cell, in the units of the moments:
 *   W = (rho, rho u, E, Er),  E = sum w |xi|^2 f0 + sum w f1 = rho|u|^2 + 1.5 rho Tt + Er,
 *   Er = sum w f1 = (dr/2) rho Tr   (monatomic: 5 unknowns, Er = 0).
 * These are the moments 1, xi, |xi|^2 (and 1 on f1) of the kinetic equation,
 * so the face fluxes are
 *   mass rho u_n;  momentum rho u u_n + (p n + sigma.n)/2;
 *   energy (E + p) u_n + (sigma.n).u + q.n + qr.n;  Er: Er u_n + qr.n,  p = rho Tt.
 * Constitutive relations of Eq. (full_constitutive): sigma = sigma_NSF(W) +
 * HoT_sigma, q = q_NSF(W) + HoT_q, the high-order terms frozen at each face
 * at the kinetic state:  everything the NSF face flux misses is carried as
 *   HoT_face = F_kin,face(f^{n+1/2}) - F_face(W^{n+1/2}),
 * F_kin the kinetic scheme's own face flux of the moments (first-order
 * upwind: sum over xi_n > 0 of w xi_n psi f of the left cell plus sum over
 * xi_n < 0 of the right cell), F_face the macroscopic face flux below without
 * HoT.  In the continuum limit this is the difference of the kinetic and NSF
 * stress and heat flux of Eq. (full_constitutive); discretely it makes the
 * macroscopic face flux at W^{n+1/2} the kinetic one, so a fixed point of the
 * kinetic iteration is a fixed point of the macroscopic solve and of GSIS.
 * NSF laws of Eq. (NSF_constitutive), Eq. (mu_kappa) in these units:
 *   sigma_NSF = -(Tt^omega/delta) (grad u + grad u^T - (2/3) div u I),
 *   q_NSF = -(k_t Tt^omega/delta) grad Tt,  qr_NSF = -(k_r Tt^omega/delta) grad Tr,
 *   monatomic k_t = 15/8 (Pr = 2/3); diatomic [k_t; k_r] = A^{-1} [5; dr] / 4.
 * Face gradients: normal derivative (X_j - X_i)/h, tangential derivatives the
 * mean of the two cells' central (one-sided at walls) gradients.
 * Convective flux: Rusanov with s = max(|u_n| + c_s), c_s = sqrt(gamma Tt / 2).
 * Boundary faces: the kinetic boundary flux of f^{n+1/2} keeps its
 * non-equilibrium part while its equilibrium part follows the iterate, in the
 * spirit of Eq. (updatef):  F_b(W^m) = F_kin + F_eq(W^m) - F_eq(W^{n+1/2}),
 * where F_eq(W) is the same face flux for the Maxwellian M(W) of the cell
 * (outgoing half of M(W), incoming wall Maxwellian with zero mass flux, or the
 * fixed inflow).  A frozen F_kin alone leaves momentum and energy fluxes that
 * need not balance, and the closed-box problem then has no steady state.
 * With wall_flux = 1 the model flux is that of the Grad-13 distributions of
 * Eq. (G13_VDF) (g13_vdf) in place of M(W):  F_b(W^m) = F_kin +
 * F_G13(W^m) - F_G13(W^{n+1/2}), the distributions built from the iterate's
 * rho, u, Tt, Tr and the stress and heat fluxes of Eq. (full_constitutive) at
 * the cell, NSF_c(W^m) + HoT_c with HoT_c the kinetic values of f^{n+1/2}
 * minus NSF_c(W^{n+1/2}) (NSF_c from the cell's central gradients), so the
 * wall flux answers the iterate's gradients next to the wall as well as its
 * state; at W^{n+1/2} the stress and heat fluxes are the kinetic ones and
 * F_b = F_kin, so a kinetic fixed point stays a fixed point.
 * Iteration: point-Jacobi on the diagonal D of Eq. (res_macro),
 *   D_i = 1/dtau_i + (1/2) sum_faces Gamma / h,  Gamma = s + C_d Tt^omega / (delta rho h),
 *   1/dtau_i = (|u| + c_s + C_d Tt^omega/(delta rho h_min)) / (CFL h_min),
 * C_d = 2 max(diffusivities) (momentum 1/2, heat k_t/1.5, rotational heat
 * k_r/(dr/2)).  Every cell takes the same pseudo-time step, D* = max_i D_i of
 * the current iterate, so that sum_i dW_i = sum_i R_i / D* = 0 and the
 * iteration conserves mass, momentum and energy exactly between walls of zero
 * flux (a local step would move total mass along the neutral direction of a
 * closed box).  The rotational relaxation -dQ/dEr = 1/(Z tau) is added to the
 * Er row of each cell.  Finally Eq. (updatef): f0 += M(W^{n+1}) - M(W^{n+1/2}),
 * f1 += (dr/2)[Tr' M(W^{n+1}) - Tr M(W^{n+1/2})], M with the translational
 * temperature (the zero-order solution of the Chapman-Enskog expansion). */
typedef struct { double rho, u[3], Tt, Tr, p, cs, E, Er; } prim_t;

typedef struct {
    int dia, nw;
    int euler;              /* Euler constitutive relations: no stress, heat flux or HoT */
    double dr, Z, delta, omega, gam, kt, kr, Cd, cfl;
} macpar;

static void macro_params(const orc_state *s, macpar *mp)
{
    const orc_cfg *c = &s->c;
    mp->dia = c->species == 1;
    mp->nw = mp->dia ? 6 : 5;
    mp->dr = c->dr;
    mp->Z = c->Zr;
    mp->delta = s->delta;
    mp->omega = c->omega;
    mp->cfl = c->macro_cfl;
    if (mp->dia) {
        double det = c->A[0] * c->A[3] - c->A[1] * c->A[2];
        double at = (c->A[3] * 5.0 - c->A[1] * c->dr) / det;
        double ar = (-c->A[2] * 5.0 + c->A[0] * c->dr) / det;
        mp->kt = at / 4.0;
        mp->kr = ar / 4.0;
        mp->gam = (5.0 + c->dr) / (3.0 + c->dr);
    } else {
        mp->kt = 15.0 / 8.0;
        mp->kr = 0.0;
        mp->gam = 5.0 / 3.0;
    }
    double nu = 0.5;
    if (mp->kt / 1.5 > nu) nu = mp->kt / 1.5;
    if (mp->dia && mp->kr / (0.5 * mp->dr) > nu) nu = mp->kr / (0.5 * mp->dr);
    mp->Cd = 2.0 * nu;
}

static void prim_of(const macpar *mp, const double *W, prim_t *P)
{
    P->rho = W[0];
    for (int a = 0; a < 3; ++a) P->u[a] = W[1 + a] / W[0];
    P->E = W[4];
    P->Er = mp->dia ? W[5] : 0.0;
    double u2 = P->u[0] * P->u[0] + P->u[1] * P->u[1] + P->u[2] * P->u[2];
    P->Tt = (2.0 / 3.0) * (P->E - P->Er - P->rho * u2) / P->rho;
    P->Tr = mp->dia ? 2.0 * P->Er / (mp->dr * P->rho) : P->Tt;
    P->p = P->rho * P->Tt;
    P->cs = sqrt(mp->gam * P->Tt / 2.0);
}

/* Central (one-sided next to non-fluid neighbours) gradient G[b*3+c] = d u_b / d x_c. */
static void cell_grad(const orc_state *s, const prim_t *P, int cell, double G[9])
{
    for (int c = 0; c < 3; ++c) {
        int nm = neighbour(s, cell, 2 * c), np = neighbour(s, cell, 2 * c + 1);
        double h = s->h[c];
        for (int b = 0; b < 3; ++b) {
            double g;
            if (nm >= 0 && np >= 0) g = (P[np].u[b] - P[nm].u[b]) / (2.0 * h);
            else if (np >= 0) g = (P[np].u[b] - P[cell].u[b]) / h;
            else if (nm >= 0) g = (P[cell].u[b] - P[nm].u[b]) / h;
            else g = 0.0;
            G[b * 3 + c] = g;
        }
    }
}

/* Central (one-sided next to non-fluid neighbours) gradients of Tt and Tr of a cell. */
static void cell_tgrad(const orc_state *s, const prim_t *P, int cell, double gt[3], double gr[3])
{
    for (int c = 0; c < 3; ++c) {
        int nm = neighbour(s, cell, 2 * c), np = neighbour(s, cell, 2 * c + 1);
        double h = s->h[c];
        const prim_t *A = &P[np >= 0 ? np : cell], *B = &P[nm >= 0 ? nm : cell];
        double den = (nm >= 0 && np >= 0) ? 2.0 * h : h;
        int none = nm < 0 && np < 0;
        gt[c] = none ? 0.0 : (A->Tt - B->Tt) / den;
        gr[c] = none ? 0.0 : (A->Tr - B->Tr) / den;
    }
}

static void ucell_grad(const orc_state *s, const prim_t *P, int i, double G[9]);
static void ucell_tgrad(const orc_state *s, const prim_t *P, int i, double gt[3], double gr[3]);

/* Stress and heat fluxes of a cell by Eq. (NSF_constitutive) from its central
 * gradients (on an unstructured mesh its least-squares gradients), sq =
 * (sigma xx yy zz xy xz yz, q, qr), mu = Tt^omega / delta. */
static void cell_nsf(const orc_state *s, const macpar *mp, const prim_t *P, int cell, double sq[12])
{
    double G[9], gt[3], gr[3];
    if (s->umesh) {
        ucell_grad(s, P, cell, G);
        ucell_tgrad(s, P, cell, gt, gr);
    } else {
        cell_grad(s, P, cell, G);
        cell_tgrad(s, P, cell, gt, gr);
    }
    double mu = pow(P[cell].Tt, mp->omega) / mp->delta;
    double div = G[0] + G[4] + G[8];
    static const int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
    for (int k = 0; k < 6; ++k) {
        int a = pa[k], b = pb[k];
        sq[k] = -mu * (G[a * 3 + b] + G[b * 3 + a] - (a == b ? (2.0 / 3.0) * div : 0.0));
    }
    for (int a = 0; a < 3; ++a) {
        sq[6 + a] = -mp->kt * mu * gt[a];
        sq[9 + a] = mp->dia ? -mp->kr * mu * gr[a] : 0.0;
    }
}

/* High-order terms of a cell for the Grad-13 wall flux: the kinetic stress and
 * heat fluxes of f^{n+1/2} (moments K) minus the cell's NSF values at
 * W^{n+1/2} (prims P), hot[12] in the order of sq. */
static void g13_cell_hot(const orc_state *s, const macpar *mp, const moms *K, const prim_t *P, int cell, double hot[12])
{
    cell_nsf(s, mp, P, cell, hot);
    for (int k = 0; k < 6; ++k) hot[k] = K->sig[k] - hot[k];
    for (int a = 0; a < 3; ++a) {
        hot[6 + a] = K->q[a] - hot[6 + a];
        hot[9 + a] = mp->dia ? K->qr[a] - hot[9 + a] : 0.0;
    }
}

/* Stress and heat fluxes of Eq. (full_constitutive) at a cell for the iterate
 * (prims P): NSF_c(W^m) + HoT_c. */
static void g13_cell_stress(const orc_state *s, const macpar *mp, const prim_t *P, int cell, const double hot[12],
                            double sq[12])
{
    cell_nsf(s, mp, P, cell, sq);
    for (int k = 0; k < 12; ++k) sq[k] += hot[k];
}

/* NSF stress column sigma_{b a} (b = x,y,z), q_a, qr_a at the face between L and
 * R = L + e_a. */
static void nsf_face(const macpar *mp, const prim_t *L, const prim_t *R, const double *gL,
                     const double *gR, int a, double h, double sigN[3], double *qN, double *qrN)
{
    double TF = 0.5 * (L->Tt + R->Tt);
    double mu = pow(TF, mp->omega) / mp->delta;
    double G[9];
    for (int b = 0; b < 3; ++b)
        for (int c = 0; c < 3; ++c)
            G[b * 3 + c] = (c == a) ? (R->u[b] - L->u[b]) / h : 0.5 * (gL[b * 3 + c] + gR[b * 3 + c]);
    double div = G[0] + G[4] + G[8];
    for (int b = 0; b < 3; ++b)
        sigN[b] = -mu * (G[b * 3 + a] + G[a * 3 + b] - (b == a ? (2.0 / 3.0) * div : 0.0));
    *qN = -mp->kt * mu * (R->Tt - L->Tt) / h;
    *qrN = mp->dia ? -mp->kr * mu * (R->Tr - L->Tr) / h : 0.0;
}

/* Flux from L to R across the face normal to axis a; hot = (sigma col, q, qr). */
static void face_flux(const macpar *mp, const prim_t *L, const prim_t *R, const double *gL,
                      const double *gR, int a, double h, const double hot[5], double F[6], double *Gam)
{
    double sigN[3] = {0, 0, 0}, qN = 0, qrN = 0;
    if (!mp->euler) nsf_face(mp, L, R, gL, gR, a, h, sigN, &qN, &qrN);
    const prim_t *S[2] = {L, R};
    double Phi[2][6], Wv[2][6];
    for (int k = 0; k < 2; ++k) {
        const prim_t *P = S[k];
        double un = P->u[a];
        Phi[k][0] = P->rho * un;
        for (int b = 0; b < 3; ++b) Phi[k][1 + b] = P->rho * P->u[b] * un + (b == a ? 0.5 * P->p : 0.0);
        Phi[k][4] = (P->E + P->p) * un;
        Phi[k][5] = P->Er * un;
        Wv[k][0] = P->rho;
        for (int b = 0; b < 3; ++b) Wv[k][1 + b] = P->rho * P->u[b];
        Wv[k][4] = P->E;
        Wv[k][5] = P->Er;
    }
    double sL = fabs(L->u[a]) + L->cs, sR = fabs(R->u[a]) + R->cs;
    double smax = sL > sR ? sL : sR;
    for (int k = 0; k < 6; ++k) F[k] = 0.5 * (Phi[0][k] + Phi[1][k]) - 0.5 * smax * (Wv[1][k] - Wv[0][k]);
    double sn[3], uF[3];
    for (int b = 0; b < 3; ++b) { sn[b] = sigN[b] + hot[b]; uF[b] = 0.5 * (L->u[b] + R->u[b]); }
    double qn = qN + hot[3], qrn = mp->dia ? qrN + hot[4] : 0.0;
    for (int b = 0; b < 3; ++b) F[1 + b] += 0.5 * sn[b];
    F[4] += sn[0] * uF[0] + sn[1] * uF[1] + sn[2] * uF[2] + qn + qrn;
    F[5] += qrn;
    double TF = 0.5 * (L->Tt + R->Tt), rF = 0.5 * (L->rho + R->rho);
    *Gam = mp->euler ? smax : smax + mp->Cd * pow(TF, mp->omega) / (mp->delta * rF * h);
}

/* Kinetic boundary flux of face (cell, d) out of the cell (O6 in the text above):
 * sum w (xi.n) psi f_face, psi = (1, xi, |xi|^2 f0 + f1, f1); f_face = f of the
 * cell for outgoing nodes and the boundary value (with rho_w recomputed from
 * this f, so the wall mass flux is exactly zero) for incoming nodes. */
static void kinetic_face_flux(const orc_state *s, int cell, int d, int bc, double F[6])
{
    const orc_cfg *c = &s->c;
    int a = d / 2;
    double sg = (d & 1) ? 1.0 : -1.0;
    double sc = face_scale(s, cell, d, bc);
    const double *f0 = s->f0 + (size_t)cell * s->nv;
    const double *f1 = s->f1 ? s->f1 + (size_t)cell * s->nv : NULL;
    nsum acc[6];
    memset(acc, 0, sizeof acc);
    for (int v = 0; v < s->nv; ++v) {
        double xi[3], w;
        node_xi(s, v, xi, &w);
        double xn = sg * xi[a];
        if (xn == 0.0) continue;
        double a0, a1;
        if (xn > 0) { a0 = f0[v]; a1 = f1 ? f1[v] : 0.0; }
        else boundary_value(c, bc, sc, xi, &a0, &a1);
        if (!f1) a1 = 0.0;
        double x2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
        double ww = w * xn;
        nadd(&acc[0], ww * a0);
        for (int b = 0; b < 3; ++b) nadd(&acc[1 + b], ww * xi[b] * a0);
        nadd(&acc[4], ww * (x2 * a0 + a1));
        nadd(&acc[5], ww * a1);
    }
    for (int k = 0; k < 6; ++k) F[k] = nval(&acc[k]);
}

/* Kinetic flux across the interior face between fluid cells L and R = L + e_a,
 * in the +a direction: sum over xi_a > 0 of w xi_a psi f_L plus sum over
 * xi_a < 0 of w xi_a psi f_R, psi = (1, xi, |xi|^2 f0 + f1, f1) (first-order
 * upwind interface values, as in the kinetic update). */
static void kinetic_interior_flux(const orc_state *s, int L, int R, int a, double F[6])
{
    const double *f0L = s->f0 + (size_t)L * s->nv, *f0R = s->f0 + (size_t)R * s->nv;
    const double *f1L = s->f1 ? s->f1 + (size_t)L * s->nv : NULL;
    const double *f1R = s->f1 ? s->f1 + (size_t)R * s->nv : NULL;
    nsum acc[6];
    memset(acc, 0, sizeof acc);
    for (int v = 0; v < s->nv; ++v) {
        double xi[3], w;
        node_xi(s, v, xi, &w);
        double xn = xi[a];
        if (xn == 0.0) continue;
        double a0 = xn > 0 ? f0L[v] : f0R[v];
        double a1 = s->f1 ? (xn > 0 ? f1L[v] : f1R[v]) : 0.0;
        double x2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
        double ww = w * xn;
        nadd(&acc[0], ww * a0);
        for (int b = 0; b < 3; ++b) nadd(&acc[1 + b], ww * xi[b] * a0);
        nadd(&acc[4], ww * (x2 * a0 + a1));
        nadd(&acc[5], ww * a1);
    }
    for (int k = 0; k < 6; ++k) F[k] = nval(&acc[k]);
}

/* Grad-13 reconstruction of a cell's distributions from its macroscopic state
 * and its stress and heat fluxes (Eq. G13_VDF), in the units above
 * (velocities in sqrt(2 R T0), sigma = 2 int (cc - |c|^2 I/3) f0,
 * q = int c |c|^2 f0, qr = int c f1).  With c = xi - u and M the Maxwellian
 * of (rho, u, Tt) (pre = (pi Tt)^{-3/2}):
 *   f0 = M [1 + sigma:cc / (rho Tt^2) + 2 (q.c) / (rho Tt^2) (2 |c|^2 / (5 Tt) - 1)],
 *   f1 = (dr/2) Tr f0 + 2 M (qr.c) / (rho Tt).
 * The printed coefficients (1/(2 rho T^2), (c^2/(5T) - 1)/(rho T^2) and
 * 1/(rho Tt)) are those of velocities in sqrt(R T0) with sigma = int (cc -
 * ..) f and q = (1/2) int c c^2 f; in the units here the forms above give
 * back rho, u, Tt, sigma, q, Tr and qr as the moments of Eq. (getmoment).
 * sq = (sigma xx yy zz xy xz yz, q, qr); sq == NULL: the Maxwellian itself. */
static void g13_vdf(const orc_cfg *c, const prim_t *P, double pre, const double *sq, const double xi[3],
                    double *f0, double *f1)
{
    double M = maxwellian_pre(P->rho, pre, P->u, P->Tt, xi);
    if (!sq) {
        *f0 = M;
        *f1 = c->species == 1 ? 0.5 * c->dr * P->Tr * M : 0.0;
        return;
    }
    double cx = xi[0] - P->u[0], cy = xi[1] - P->u[1], cz = xi[2] - P->u[2];
    double c2 = cx * cx + cy * cy + cz * cz;
    double rT2 = P->rho * P->Tt * P->Tt;
    double scc = sq[0] * cx * cx + sq[1] * cy * cy + sq[2] * cz * cz
               + 2.0 * (sq[3] * cx * cy + sq[4] * cx * cz + sq[5] * cy * cz);
    double qc = sq[6] * cx + sq[7] * cy + sq[8] * cz;
    double b = 1.0 + scc / rT2 + 2.0 * qc / rT2 * (2.0 * c2 / (5.0 * P->Tt) - 1.0);
    *f0 = M * b;
    if (c->species == 1) {
        double qrc = sq[9] * cx + sq[10] * cy + sq[11] * cz;
        *f1 = 0.5 * c->dr * P->Tr * (*f0) + 2.0 * M * qrc / (P->rho * P->Tt);
    } else {
        *f1 = 0.0;
    }
}

/* The flux of a boundary face when the cell holds the Maxwellian of W
 * (f1 = (dr/2) Tr M) -- F_eq -- or, given sq, the Grad-13 distributions of
 * g13_vdf -- F_G13, Eq. (GSIS-DVM-flux) -- with the same boundary rule: the
 * cell's distributions at the outgoing nodes, the boundary value at the
 * incoming ones (a wall's density from zero net mass flux). */
static void model_face_flux(const orc_state *s, const prim_t *P, const double *sq, int d, int bc, double F[6])
{
    const orc_cfg *c = &s->c;
    int a = d / 2;
    double sg = (d & 1) ? 1.0 : -1.0;
    int dia = c->species == 1;
    double sc = c->bc_rho[bc];
    const double pc = pow(M_PI * P->Tt, -1.5);
    const double *Mb = s->mbw + (size_t)bc * s->nv;
    /* the cell's distributions at the outgoing nodes, evaluated once */
    double *Mc = malloc(sizeof(double) * (size_t)s->nv);
    double *Mc1 = malloc(sizeof(double) * (size_t)s->nv);
    for (int v = 0; v < s->nv; ++v) {
        double xi[3], w;
        node_xi(s, v, xi, &w);
        Mc[v] = Mc1[v] = 0.0;
        if (sg * xi[a] > 0) g13_vdf(c, P, pc, sq, xi, &Mc[v], &Mc1[v]);
    }
    if (c->bc_kind[bc] == ORC_WALL) {
        nsum out = {0, 0};
        for (int v = 0; v < s->nv; ++v) {
            double xi[3], w;
            node_xi(s, v, xi, &w);
            double xn = sg * xi[a];
            if (xn > 0) nadd(&out, w * xn * Mc[v]);
        }
        sc = nval(&out) / s->in_half[d][bc];
    }
    nsum acc[6];
    memset(acc, 0, sizeof acc);
    for (int v = 0; v < s->nv; ++v) {
        double xi[3], w;
        node_xi(s, v, xi, &w);
        double xn = sg * xi[a];
        if (xn == 0.0) continue;
        double a0, a1;
        if (xn > 0) {
            a0 = Mc[v];
            a1 = Mc1[v];
        } else {
            /* the boundary value sc M(1, u_b, T_b) (f1: (dr/2) T_b times it) */
            a0 = sc * Mb[v];
            a1 = dia ? 0.5 * c->dr * c->bc_T[bc] * a0 : 0.0;
        }
        double x2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
        double ww = w * xn;
        nadd(&acc[0], ww * a0);
        for (int b = 0; b < 3; ++b) nadd(&acc[1 + b], ww * xi[b] * a0);
        nadd(&acc[4], ww * (x2 * a0 + a1));
        nadd(&acc[5], ww * a1);
    }
    for (int k = 0; k < 6; ++k) F[k] = nval(&acc[k]);
    free(Mc);
    free(Mc1);
}


/* The macroscopic solve from the kinetic moments K[cell] of f^{n+1/2}, the
 * kinetic boundary fluxes Fkin[cell][6][6] (out of the cell through each
 * boundary face) and the kinetic interior fluxes Fint[cell][3][6] (through
 * the face to the +a neighbour, where that is a fluid cell) (both unused for
 * euler), iters point-Jacobi iterations; returns
 * the primitive variables of W^{n+1} in Pn[cell] and keeps W^{n+1} in
 * s->lastW.  Sets s->status to -5 on a non-physical result.
 * euler = 1: the same iteration with the Euler constitutive relations (no
 * stress, heat flux or HoT, no diffusive part in Gamma and dtau) and the
 * boundary flux of the iterate's own Maxwellian, F_b(W^m) = F_eq(W^m): the
 * initial-field computation of Alg. 1, line 1. */
static int macro_solve(orc_state *s, const moms *K, const double *Fkin, const double *Fint, int iters, int euler,
                       prim_t *P)
{
    const orc_cfg *c = &s->c;
    macpar mp;
    macro_params(s, &mp);
    mp.euler = euler;
    int ncell = s->ncell, nw = mp.nw;
    double hmin = s->h[0];
    if (s->h[1] < hmin) hmin = s->h[1];
    if (s->h[2] < hmin) hmin = s->h[2];
    double *W = calloc((size_t)ncell * 6, sizeof(double));
    double *Fb = calloc((size_t)ncell * 36, sizeof(double));
    double *fix = calloc((size_t)ncell * 18, sizeof(double));   /* HoT_face per (cell, +a face), 6 each */
    static const double nohot[5] = {0, 0, 0, 0, 0};
    double *grad = calloc((size_t)ncell * 9, sizeof(double));
    double *R = calloc((size_t)ncell * 6, sizeof(double));
    double *Dc = calloc((size_t)ncell, sizeof(double));
    double *Src = calloc((size_t)ncell, sizeof(double));
    /* Grad-13 boundary flux: the high-order terms of each cell with a boundary
     * face, HoT_c = (sigma, q, qr)(f^{n+1/2}) - NSF_c(W^{n+1/2}), so that the
     * stress and heat fluxes of the iterate, NSF_c(W^m) + HoT_c (Eq.
     * full_constitutive at the cell), are the kinetic ones at W^{n+1/2} */
    const int g13 = c->wall_flux == 1 && !euler;
    double *hotc = g13 ? calloc((size_t)ncell * 12, sizeof(double)) : NULL;

    /* the starting W from the kinetic moments, and the fixed boundary fluxes */
    for (int cell = 0; cell < ncell; ++cell) {
        if (s->solid[cell]) continue;
        const moms *m = &K[cell];
        double u2 = m->u[0] * m->u[0] + m->u[1] * m->u[1] + m->u[2] * m->u[2];
        double *w = W + (size_t)cell * 6;
        w[0] = m->rho;
        for (int a = 0; a < 3; ++a) w[1 + a] = m->rho * m->u[a];
        double Er = mp.dia ? 0.5 * c->dr * m->rho * m->Tr : 0.0;
        w[4] = m->rho * u2 + 1.5 * m->rho * m->Tt + Er;
        w[5] = Er;
        if (!euler) memcpy(Fb + (size_t)cell * 36, Fkin + (size_t)cell * 36, 36 * sizeof(double));
    }
    /* HoT at interior faces (cell, cell + e_a), from W^{n+1/2} */
    for (int cell = 0; cell < ncell; ++cell)
        if (!s->solid[cell]) prim_of(&mp, W + (size_t)cell * 6, &P[cell]);
    if (g13) {
        for (int cell = 0; cell < ncell; ++cell) {
            if (s->solid[cell]) continue;
            int nbnd = 0;
            for (int d = 0; d < 6; ++d) nbnd += neighbour(s, cell, d) < 0;
            if (!nbnd) continue;
            g13_cell_hot(s, &mp, &K[cell], P, cell, hotc + (size_t)cell * 12);
        }
    }
    /* fixed part of the boundary fluxes: F_kin - F_model(W^{n+1/2}) (zero for Euler) */
    #pragma omp parallel for schedule(dynamic, 16)
    for (int cell = 0; cell < ncell; ++cell) {
        if (s->solid[cell] || euler) continue;
        double sq[12];
        if (g13) g13_cell_stress(s, &mp, P, cell, hotc + (size_t)cell * 12, sq);
        for (int d = 0; d < 6; ++d) {
            int n = neighbour(s, cell, d);
            if (n >= 0) continue;
            double Fe[6];
            model_face_flux(s, &P[cell], g13 ? sq : NULL, d, -1 - n, Fe);
            for (int k = 0; k < 6; ++k) Fb[(size_t)cell * 36 + d * 6 + k] -= Fe[k];
        }
    }
    for (int cell = 0; cell < ncell; ++cell)
        if (!s->solid[cell]) cell_grad(s, P, cell, grad + (size_t)cell * 9);
    for (int cell = 0; cell < ncell; ++cell) {
        if (s->solid[cell] || euler) continue;    /* no HoT for Euler */
        for (int a = 0; a < 3; ++a) {
            int nb = neighbour(s, cell, 2 * a + 1);
            if (nb < 0) continue;
            double F[6], Gam;
            face_flux(&mp, &P[cell], &P[nb], grad + (size_t)cell * 9, grad + (size_t)nb * 9, a, s->h[a], nohot, F, &Gam);
            double *fx = fix + (size_t)cell * 18 + a * 6;
            const double *fk = Fint + (size_t)cell * 18 + a * 6;
            for (int k = 0; k < 6; ++k) fx[k] = fk[k] - F[k];
            if (!mp.dia) fx[5] = 0.0;
        }
    }
    /* point-Jacobi iterations */
    for (int it = 0; it < iters; ++it) {
        for (int cell = 0; cell < ncell; ++cell)
            if (!s->solid[cell]) prim_of(&mp, W + (size_t)cell * 6, &P[cell]);
        for (int cell = 0; cell < ncell; ++cell)
            if (!s->solid[cell]) cell_grad(s, P, cell, grad + (size_t)cell * 9);
        #pragma omp parallel for schedule(dynamic, 16)
        for (int cell = 0; cell < ncell; ++cell) {
            if (s->solid[cell]) continue;
            const prim_t *Pi = &P[cell];
            double res[6] = {0, 0, 0, 0, 0, 0}, sumG = 0;
            for (int d = 0; d < 6; ++d) {
                int a = d / 2;
                double h = s->h[a];
                int n = neighbour(s, cell, d);
                double F[6], out[6], Gam;
                if (n >= 0) {
                    int L = (d & 1) ? cell : n, Rr = (d & 1) ? n : cell;
                    face_flux(&mp, &P[L], &P[Rr], grad + (size_t)L * 9, grad + (size_t)Rr * 9, a, h, nohot, F, &Gam);
                    const double *fx = fix + (size_t)L * 18 + a * 6;
                    for (int k = 0; k < 6; ++k) out[k] = (d & 1) ? F[k] + fx[k] : -(F[k] + fx[k]);
                } else {
                    double Fe[6], sq[12];
                    if (g13) g13_cell_stress(s, &mp, P, cell, hotc + (size_t)cell * 12, sq);
                    model_face_flux(s, Pi, g13 ? sq : NULL, d, -1 - n, Fe);
                    for (int k = 0; k < 6; ++k) out[k] = Fb[(size_t)cell * 36 + d * 6 + k] + Fe[k];
                    Gam = fabs(Pi->u[a]) + Pi->cs;
                    if (!euler) Gam += mp.Cd * pow(Pi->Tt, mp.omega) / (mp.delta * Pi->rho * h);
                }
                for (int k = 0; k < nw; ++k) res[k] -= out[k] / h;
                sumG += Gam / h;
            }
            double invtau = mp.delta * Pi->rho * pow(Pi->Tt, 1.0 - mp.omega);
            if (mp.dia) {
                double T = (3.0 * Pi->Tt + mp.dr * Pi->Tr) / (3.0 + mp.dr);
                res[5] += 0.5 * mp.dr * Pi->rho * (T - Pi->Tr) * invtau / mp.Z;
            }
            double umag = sqrt(Pi->u[0] * Pi->u[0] + Pi->u[1] * Pi->u[1] + Pi->u[2] * Pi->u[2]);
            double vis = euler ? 0.0 : mp.Cd * pow(Pi->Tt, mp.omega) / (mp.delta * Pi->rho * hmin);
            double idt = (umag + Pi->cs + vis) / (mp.cfl * hmin);
            double *r = R + (size_t)cell * 6;
            for (int k = 0; k < 6; ++k) r[k] = res[k];
            Dc[cell] = idt + 0.5 * sumG;
            Src[cell] = mp.dia ? invtau / mp.Z : 0.0;
        }
        double Dmax = 0.0;
        for (int cell = 0; cell < ncell; ++cell)
            if (!s->solid[cell] && Dc[cell] > Dmax) Dmax = Dc[cell];
        for (int cell = 0; cell < ncell; ++cell) {
            if (s->solid[cell]) continue;
            double *w = W + (size_t)cell * 6;
            const double *r = R + (size_t)cell * 6;
            for (int k = 0; k < 5; ++k) w[k] += r[k] / Dmax;
            if (mp.dia) w[5] += r[5] / (Dmax + Src[cell]);
        }
    }
    int bad = 0;
    for (int cell = 0; cell < ncell; ++cell) {
        if (s->solid[cell]) continue;
        prim_of(&mp, W + (size_t)cell * 6, &P[cell]);
        if (!(P[cell].rho > 0) || !(P[cell].Tt > 0) || !isfinite(P[cell].E)) bad = 1;
    }
    if (bad) s->status = -5;
    if (!s->lastW) s->lastW = malloc(sizeof(double) * (size_t)ncell * 6);
    memcpy(s->lastW, W, sizeof(double) * (size_t)ncell * 6);
    free(W); free(Fb); free(fix); free(grad); free(R); free(Dc); free(Src); free(hotc);
    return s->status;
}

/* ------------------------------------- unstructured macroscopic solve -- */
/* The GSIS-II correction on an unstructured mesh: the same equations and
 * iteration as macro_solve, written for faces of any normal n (out of the
 * owner), area S and cells of volume V, with
 *  - the velocity gradient of a cell by least squares over its face
 *    neighbours, G minimising sum_j |u_j - u_i - G (x_j - x_i)|^2: G = B A^+,
 *    A = sum_j d_j d_j^T, B = sum_j (u_j - u_i) d_j^T, A^+ the inverse on the
 *    range of A (Jacobi eigen-decomposition; eigenvalues below 1e-12 of the
 *    largest dropped), so a direction without neighbours gets no gradient
 *    (on whole hexahedra: the central, next to a boundary one-sided,
 *    difference of macro_solve);
 *  - at a face between L and R (d = x_R - x_L): the face gradient is the mean
 *    of the two cells' plus the correction that makes its component along d
 *    the two-cell difference, G_f = Gm + [(u_R - u_L)/|d| - Gm d/|d|] d^T/|d|,
 *    the normal heat fluxes -k mu (T_R - T_L) / h and h = d . n (on
 *    hexahedra: the normal difference and mean tangential gradients of
 *    macro_solve);
 *  - Gamma = s + C_d Tt^omega / (delta rho h), h = d . n inside and twice the
 *    distance along n from the cell centroid to the face centroid on a
 *    boundary face; h_min of the pseudo time step the smallest of these;
 *  - face fluxes per unit area times S / V in the residual and the diagonal,
 *    D_i = 1/dtau_i + (1/2) sum_faces Gamma S / V;
 *  - the high-order terms of reading "face-consistent HoT": at every face the
 *    kinetic scheme's flux of f^{n+1/2} (first-order upwind values across
 *    the face's own normal) minus the macroscopic flux of W^{n+1/2}. */
static void sym3_pinv(const double A[9], double Pi[9])
{
    double a[3][3], v[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) a[i][j] = A[i * 3 + j];
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
        if (off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (a[p][q] == 0.0) continue;
                double th = 0.5 * (a[q][q] - a[p][p]) / a[p][q];
                double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < 3; ++k) {   /* A <- A J */
                    double x = a[k][p], y = a[k][q];
                    a[k][p] = cs * x - sn * y;
                    a[k][q] = sn * x + cs * y;
                }
                for (int k = 0; k < 3; ++k) {   /* A <- J^T A */
                    double x = a[p][k], y = a[q][k];
                    a[p][k] = cs * x - sn * y;
                    a[q][k] = sn * x + cs * y;
                }
                for (int k = 0; k < 3; ++k) {   /* V <- V J */
                    double x = v[k][p], y = v[k][q];
                    v[k][p] = cs * x - sn * y;
                    v[k][q] = sn * x + cs * y;
                }
            }
    }
    double emax = fmax(fabs(a[0][0]), fmax(fabs(a[1][1]), fabs(a[2][2])));
    double inv[3];
    for (int k = 0; k < 3; ++k) inv[k] = (emax > 0 && a[k][k] > 1e-12 * emax) ? 1.0 / a[k][k] : 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += v[i][k] * inv[k] * v[j][k];
            Pi[i * 3 + j] = acc;
        }
}

static void ucell_grad(const orc_state *s, const prim_t *P, int i, double G[9])
{
    double A[9] = {0}, B[9] = {0}, Ai[9];
    const double *xi = s->ucen + (size_t)i * 3;
    for (int e = s->cf_off[i]; e < s->cf_off[i + 1]; ++e) {
        double n[3], sv;
        int j;
        uface_of(s, i, s->cf[e], n, &sv, &j);
        if (j < 0) continue;
        const double *xj = s->ucen + (size_t)j * 3;
        double d[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) {
                A[b * 3 + c] += d[b] * d[c];
                B[b * 3 + c] += (P[j].u[b] - P[i].u[b]) * d[c];
            }
    }
    sym3_pinv(A, Ai);
    for (int b = 0; b < 3; ++b)
        for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += B[b * 3 + k] * Ai[k * 3 + c];
            G[b * 3 + c] = acc;
        }
}

/* Least-squares gradients of Tt and Tr of cell i, with the weights of
 * ucell_grad. */
static void ucell_tgrad(const orc_state *s, const prim_t *P, int i, double gt[3], double gr[3])
{
    double A[9] = {0}, bt[3] = {0}, br[3] = {0}, Ai[9];
    const double *xi = s->ucen + (size_t)i * 3;
    for (int e = s->cf_off[i]; e < s->cf_off[i + 1]; ++e) {
        double n[3], sv;
        int j;
        uface_of(s, i, s->cf[e], n, &sv, &j);
        if (j < 0) continue;
        const double *xj = s->ucen + (size_t)j * 3;
        double d[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
        for (int b = 0; b < 3; ++b) {
            for (int c = 0; c < 3; ++c) A[b * 3 + c] += d[b] * d[c];
            bt[b] += (P[j].Tt - P[i].Tt) * d[b];
            br[b] += (P[j].Tr - P[i].Tr) * d[b];
        }
    }
    sym3_pinv(A, Ai);
    for (int c = 0; c < 3; ++c) {
        double at = 0, ar = 0;
        for (int k = 0; k < 3; ++k) {
            at += bt[k] * Ai[k * 3 + c];
            ar += br[k] * Ai[k * 3 + c];
        }
        gt[c] = at;
        gr[c] = ar;
    }
}

/* Flux from L to R across a face of unit normal n (out of L), d = x_R - x_L,
 * hot = HoT of the six flux components added as given. */
static void uface_flux(const macpar *mp, const prim_t *L, const prim_t *R, const double *gL, const double *gR,
                       const double n[3], const double d[3], const double hot[6], double F[6], double *Gam)
{
    double h = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];
    double sN[3] = {0, 0, 0}, qN = 0, qrN = 0;
    double TF = 0.5 * (L->Tt + R->Tt);
    if (!mp->euler) {
        double mu = pow(TF, mp->omega) / mp->delta;
        double dl = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double e[3] = {d[0] / dl, d[1] / dl, d[2] / dl};
        double G[9];
        for (int b = 0; b < 3; ++b) {
            double gm[3], gd = 0;
            for (int c = 0; c < 3; ++c) { gm[c] = 0.5 * (gL[b * 3 + c] + gR[b * 3 + c]); gd += gm[c] * e[c]; }
            double corr = (R->u[b] - L->u[b]) / dl - gd;
            for (int c = 0; c < 3; ++c) G[b * 3 + c] = gm[c] + corr * e[c];
        }
        double div = G[0] + G[4] + G[8];
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int c = 0; c < 3; ++c) acc += (G[b * 3 + c] + G[c * 3 + b]) * n[c];
            sN[b] = -mu * (acc - (2.0 / 3.0) * div * n[b]);
        }
        qN = -mp->kt * mu * (R->Tt - L->Tt) / h;
        qrN = mp->dia ? -mp->kr * mu * (R->Tr - L->Tr) / h : 0.0;
    }
    const prim_t *S[2] = {L, R};
    double Phi[2][6], Wv[2][6], un[2];
    for (int k = 0; k < 2; ++k) {
        const prim_t *Pk = S[k];
        un[k] = Pk->u[0] * n[0] + Pk->u[1] * n[1] + Pk->u[2] * n[2];
        Phi[k][0] = Pk->rho * un[k];
        for (int b = 0; b < 3; ++b) Phi[k][1 + b] = Pk->rho * Pk->u[b] * un[k] + 0.5 * Pk->p * n[b];
        Phi[k][4] = (Pk->E + Pk->p) * un[k];
        Phi[k][5] = Pk->Er * un[k];
        Wv[k][0] = Pk->rho;
        for (int b = 0; b < 3; ++b) Wv[k][1 + b] = Pk->rho * Pk->u[b];
        Wv[k][4] = Pk->E;
        Wv[k][5] = Pk->Er;
    }
    double sL = fabs(un[0]) + L->cs, sR = fabs(un[1]) + R->cs;
    double smax = sL > sR ? sL : sR;
    for (int k = 0; k < 6; ++k) F[k] = 0.5 * (Phi[0][k] + Phi[1][k]) - 0.5 * smax * (Wv[1][k] - Wv[0][k]);
    double uF[3];
    for (int b = 0; b < 3; ++b) uF[b] = 0.5 * (L->u[b] + R->u[b]);
    for (int b = 0; b < 3; ++b) F[1 + b] += 0.5 * sN[b];
    F[4] += sN[0] * uF[0] + sN[1] * uF[1] + sN[2] * uF[2] + qN + qrN;
    F[5] += qrN;
    for (int k = 0; k < 6; ++k) F[k] += hot[k];
    double rF = 0.5 * (L->rho + R->rho);
    *Gam = mp->euler ? smax : smax + mp->Cd * pow(TF, mp->omega) / (mp->delta * rF * h);
}

/* The kinetic flux of face f out of its owner: sum w (xi.n) psi f_face with
 * psi = (1, xi, |xi|^2 f0 + f1, f1), f_face the upwind cell's value inside;
 * on a boundary face the owner's value going out and the boundary value
 * coming in (wall density from this f, zero mass flux). */
static void ukinetic_face_flux(const orc_state *s, int f, double F[6])
{
    const orc_cfg *c = &s->c;
    int L = s->ufc[2 * f], R = s->ufc[2 * f + 1];
    const double *g = s->ufg + (size_t)f * 4;
    const double *f0L = s->f0 + (size_t)L * s->nv, *f1L = s->f1 ? s->f1 + (size_t)L * s->nv : NULL;
    const double *f0R = R >= 0 ? s->f0 + (size_t)R * s->nv : NULL;
    const double *f1R = (R >= 0 && s->f1) ? s->f1 + (size_t)R * s->nv : NULL;
    int bc = R < 0 ? -1 - R : 0;
    double sc = R < 0 ? uface_scale(s, f) : 0.0;
    nsum acc[6];
    memset(acc, 0, sizeof acc);
    for (int v = 0; v < s->nv; ++v) {
        double xi[3], w;
        node_xi(s, v, xi, &w);
        double xn = xi[0] * g[1] + xi[1] * g[2] + xi[2] * g[3];
        if (xn == 0.0) continue;
        double a0, a1;
        if (xn > 0) {
            a0 = f0L[v];
            a1 = f1L ? f1L[v] : 0.0;
        } else if (R >= 0) {
            a0 = f0R[v];
            a1 = f1R ? f1R[v] : 0.0;
        } else {
            boundary_value(c, bc, sc, xi, &a0, &a1);
            if (!s->f1) a1 = 0.0;
        }
        double x2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
        double ww = w * xn;
        nadd(&acc[0], ww * a0);
        for (int b = 0; b < 3; ++b) nadd(&acc[1 + b], ww * xi[b] * a0);
        nadd(&acc[4], ww * (x2 * a0 + a1));
        nadd(&acc[5], ww * a1);
    }
    for (int k = 0; k < 6; ++k) F[k] = nval(&acc[k]);
}

/* F_eq of boundary face f: its flux when the owner holds the Maxwellian of P
 * (f1 = (dr/2) Tr M), with the boundary rule of the face. */
static void umodel_face_flux(const orc_state *s, const prim_t *P, const double *sq, int f, double F[6])
{
    const orc_cfg *c = &s->c;
    const double *g = s->ufg + (size_t)f * 4;
    int bc = -1 - s->ufc[2 * f + 1], dia = c->species == 1;
    const double pc = pow(M_PI * P->Tt, -1.5);
    const double *Mb = s->mbw + (size_t)bc * s->nv;
    double sc = c->bc_rho[bc];
    if (c->bc_kind[bc] == ORC_WALL) {
        nsum out = {0, 0}, in = {0, 0};
        for (int v = 0; v < s->nv; ++v) {
            double xi[3], w, o0, o1;
            node_xi(s, v, xi, &w);
            double xn = xi[0] * g[1] + xi[1] * g[2] + xi[2] * g[3];
            if (xn > 0) {
                g13_vdf(c, P, pc, sq, xi, &o0, &o1);
                nadd(&out, w * xn * o0);
            } else if (xn < 0) {
                nadd(&in, w * (-xn) * Mb[v]);
            }
        }
        sc = nval(&out) / nval(&in);
    }
    nsum acc[6];
    memset(acc, 0, sizeof acc);
    for (int v = 0; v < s->nv; ++v) {
        double xi[3], w;
        node_xi(s, v, xi, &w);
        double xn = xi[0] * g[1] + xi[1] * g[2] + xi[2] * g[3];
        if (xn == 0.0) continue;
        double a0, a1;
        if (xn > 0) {
            g13_vdf(c, P, pc, sq, xi, &a0, &a1);
        } else {
            a0 = sc * Mb[v];
            a1 = dia ? 0.5 * c->dr * c->bc_T[bc] * a0 : 0.0;
        }
        double x2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
        double ww = w * xn;
        nadd(&acc[0], ww * a0);
        for (int b = 0; b < 3; ++b) nadd(&acc[1 + b], ww * xi[b] * a0);
        nadd(&acc[4], ww * (x2 * a0 + a1));
        nadd(&acc[5], ww * a1);
    }
    for (int k = 0; k < 6; ++k) F[k] = nval(&acc[k]);
}

/* h of face f: d . n between the two centroids inside, twice the distance
 * along n from the owner's centroid to the face centroid on the boundary. */
static double uface_h(const orc_state *s, int f, double d[3])
{
    const double *g = s->ufg + (size_t)f * 4;
    int L = s->ufc[2 * f], R = s->ufc[2 * f + 1];
    const double *xL = s->ucen + (size_t)L * 3;
    const double *xR = R >= 0 ? s->ucen + (size_t)R * 3 : s->ufcen + (size_t)f * 3;
    double k = R >= 0 ? 1.0 : 2.0;
    for (int a = 0; a < 3; ++a) d[a] = k * (xR[a] - xL[a]);
    return d[0] * g[1] + d[1] * g[2] + d[2] * g[3];
}

static int umacro_solve(orc_state *s, const moms *K, int iters, int euler, prim_t *P)
{
    const orc_cfg *c = &s->c;
    macpar mp;
    macro_params(s, &mp);
    mp.euler = euler;
    int ncell = s->ncell, nw = mp.nw, nf = s->nface;
    static const double nohot[6] = {0, 0, 0, 0, 0, 0};
    double *W = calloc((size_t)ncell * 6, sizeof(double));
    double *fix = calloc((size_t)nf * 6, sizeof(double));   /* HoT of interior faces, fixed part of boundary faces */
    double *grad = calloc((size_t)ncell * 9, sizeof(double));
    double *R = calloc((size_t)ncell * 6, sizeof(double));
    double *Dc = calloc((size_t)ncell, sizeof(double));
    double *Src = calloc((size_t)ncell, sizeof(double));
    /* Grad-13 wall flux: the high-order terms of the cells with a boundary
     * face, as in macro_solve */
    const int g13 = c->wall_flux == 1 && !euler;
    double *hotc = g13 ? calloc((size_t)ncell * 12, sizeof(double)) : NULL;
    double hmin = INFINITY;
    for (int f = 0; f < nf; ++f) {
        double d[3], h = uface_h(s, f, d);
        if (h < hmin) hmin = h;
    }
    for (int cell = 0; cell < ncell; ++cell) {
        const moms *m = &K[cell];
        double u2 = m->u[0] * m->u[0] + m->u[1] * m->u[1] + m->u[2] * m->u[2];
        double *w = W + (size_t)cell * 6;
        w[0] = m->rho;
        for (int a = 0; a < 3; ++a) w[1 + a] = m->rho * m->u[a];
        double Er = mp.dia ? 0.5 * c->dr * m->rho * m->Tr : 0.0;
        w[4] = m->rho * u2 + 1.5 * m->rho * m->Tt + Er;
        w[5] = Er;
        prim_of(&mp, w, &P[cell]);
    }
    for (int cell = 0; cell < ncell; ++cell) ucell_grad(s, P, cell, grad + (size_t)cell * 9);
    for (int f = 0; g13 && f < nf; ++f)
        if (s->ufc[2 * f + 1] < 0) {
            int L = s->ufc[2 * f];
            g13_cell_hot(s, &mp, &K[L], P, L, hotc + (size_t)L * 12);
        }
    /* fixed parts: F_kin(f^{n+1/2}) - F(W^{n+1/2}) at every face (zero for
     * Euler: no high-order terms, the boundary flux of the iterate's own
     * Maxwellian) */
    #pragma omp parallel for schedule(dynamic, 16)
    for (int f = 0; f < nf * !euler; ++f) {
        int L = s->ufc[2 * f], Rr = s->ufc[2 * f + 1];
        double Fk[6], Fm[6], Gam, d[3];
        ukinetic_face_flux(s, f, Fk);
        if (Rr >= 0) {
            uface_h(s, f, d);
            uface_flux(&mp, &P[L], &P[Rr], grad + (size_t)L * 9, grad + (size_t)Rr * 9, s->ufg + (size_t)f * 4 + 1, d,
                       nohot, Fm, &Gam);
        } else {
            double sq[12];
            if (g13) g13_cell_stress(s, &mp, P, L, hotc + (size_t)L * 12, sq);
            umodel_face_flux(s, &P[L], g13 ? sq : NULL, f, Fm);
        }
        for (int k = 0; k < 6; ++k) fix[(size_t)f * 6 + k] = Fk[k] - Fm[k];
        if (!mp.dia && Rr >= 0) fix[(size_t)f * 6 + 5] = 0.0;
    }
    double *Ff = calloc((size_t)nf * 7, sizeof(double));   /* face flux (owner -> other) and Gamma of an iterate */
    for (int it = 0; it < iters; ++it) {
        for (int cell = 0; cell < ncell; ++cell) prim_of(&mp, W + (size_t)cell * 6, &P[cell]);
        for (int cell = 0; cell < ncell; ++cell) ucell_grad(s, P, cell, grad + (size_t)cell * 9);
        #pragma omp parallel for schedule(dynamic, 16)
        for (int f = 0; f < nf; ++f) {
            int L = s->ufc[2 * f], Rr = s->ufc[2 * f + 1];
            double *o = Ff + (size_t)f * 7, d[3];
            double h = uface_h(s, f, d);
            if (Rr >= 0) {
                uface_flux(&mp, &P[L], &P[Rr], grad + (size_t)L * 9, grad + (size_t)Rr * 9, s->ufg + (size_t)f * 4 + 1,
                           d, fix + (size_t)f * 6, o, &o[6]);
            } else {
                double Fe[6], sq[12];
                if (g13) g13_cell_stress(s, &mp, P, L, hotc + (size_t)L * 12, sq);
                umodel_face_flux(s, &P[L], g13 ? sq : NULL, f, Fe);
                for (int k = 0; k < 6; ++k) o[k] = fix[(size_t)f * 6 + k] + Fe[k];
                const double *g = s->ufg + (size_t)f * 4;
                const prim_t *Pi = &P[L];
                double un = Pi->u[0] * g[1] + Pi->u[1] * g[2] + Pi->u[2] * g[3];
                o[6] = fabs(un) + Pi->cs + (euler ? 0.0 : mp.Cd * pow(Pi->Tt, mp.omega) / (mp.delta * Pi->rho * h));
            }
        }
        #pragma omp parallel for schedule(dynamic, 16)
        for (int cell = 0; cell < ncell; ++cell) {
            const prim_t *Pi = &P[cell];
            double res[6] = {0, 0, 0, 0, 0, 0}, sumG = 0;
            for (int e = s->cf_off[cell]; e < s->cf_off[cell + 1]; ++e) {
                int f = s->cf[e] >> 1, side = s->cf[e] & 1;
                const double *o = Ff + (size_t)f * 7;
                double sv = s->ufg[(size_t)f * 4] / s->uvol[cell];
                for (int k = 0; k < nw; ++k) res[k] -= (side ? -o[k] : o[k]) * sv;
                sumG += o[6] * sv;
            }
            double invtau = mp.delta * Pi->rho * pow(Pi->Tt, 1.0 - mp.omega);
            if (mp.dia) {
                double T = (3.0 * Pi->Tt + mp.dr * Pi->Tr) / (3.0 + mp.dr);
                res[5] += 0.5 * mp.dr * Pi->rho * (T - Pi->Tr) * invtau / mp.Z;
            }
            double umag = sqrt(Pi->u[0] * Pi->u[0] + Pi->u[1] * Pi->u[1] + Pi->u[2] * Pi->u[2]);
            double vis = euler ? 0.0 : mp.Cd * pow(Pi->Tt, mp.omega) / (mp.delta * Pi->rho * hmin);
            double idt = (umag + Pi->cs + vis) / (mp.cfl * hmin);
            double *r = R + (size_t)cell * 6;
            for (int k = 0; k < 6; ++k) r[k] = res[k];
            Dc[cell] = idt + 0.5 * sumG;
            Src[cell] = mp.dia ? invtau / mp.Z : 0.0;
        }
        double Dmax = 0.0;
        for (int cell = 0; cell < ncell; ++cell)
            if (Dc[cell] > Dmax) Dmax = Dc[cell];
        for (int cell = 0; cell < ncell; ++cell) {
            double *w = W + (size_t)cell * 6;
            const double *r = R + (size_t)cell * 6;
            for (int k = 0; k < 5; ++k) w[k] += r[k] / Dmax;
            if (mp.dia) w[5] += r[5] / (Dmax + Src[cell]);
        }
    }
    int bad = 0;
    for (int cell = 0; cell < ncell; ++cell) {
        prim_of(&mp, W + (size_t)cell * 6, &P[cell]);
        if (!(P[cell].rho > 0) || !(P[cell].Tt > 0) || !isfinite(P[cell].E)) bad = 1;
    }
    if (bad) s->status = -5;
    if (!s->lastW) s->lastW = malloc(sizeof(double) * (size_t)ncell * 6);
    memcpy(s->lastW, W, sizeof(double) * (size_t)ncell * 6);
    free(W); free(fix); free(grad); free(R); free(Dc); free(Src); free(Ff); free(hotc);
    return s->status;
}

/* gsis_correct on the stored VDF: kinetic moments and boundary fluxes of
 * f^{n+1/2}, the macroscopic solve, then Eq. (updatef):
 * f0 += M(W^{n+1}) - M(W^{n+1/2}), f1 += (dr/2)[Tr' M(W^{n+1}) - Tr M(W^{n+1/2})],
 * M with the translational temperature (the zero-order solution of the
 * Chapman-Enskog expansion). */
static int gsis_correct_mode(orc_state *s, int iters, int euler)
{
    /* unstructured mesh: the correction needs the centroids */
    if (s->umesh && !s->ucen) return -2;
    const orc_cfg *c = &s->c;
    int ncell = s->ncell, dia = c->species == 1;
    moms *K = calloc((size_t)ncell, sizeof(moms));
    double *Fkin = s->umesh ? NULL : calloc((size_t)ncell * 36, sizeof(double));
    double *Fint = s->umesh ? NULL : calloc((size_t)ncell * 18, sizeof(double));
    prim_t *P = calloc((size_t)ncell, sizeof(prim_t));
    #pragma omp parallel for schedule(dynamic, 16)
    for (int cell = 0; cell < ncell; ++cell) {
        if (s->solid[cell]) continue;
        cell_moments(s, cell, &K[cell]);
        for (int d = 0; d < 6 && !s->umesh; ++d) {
            int n = neighbour(s, cell, d);
            if (n < 0 && !euler) kinetic_face_flux(s, cell, d, -1 - n, Fkin + (size_t)cell * 36 + d * 6);
            if (n >= 0 && (d & 1) && !euler) kinetic_interior_flux(s, cell, n, d / 2, Fint + (size_t)cell * 18 + (d / 2) * 6);
        }
    }
    if (s->umesh) umacro_solve(s, K, iters, euler, P);
    else macro_solve(s, K, Fkin, Fint, iters, euler, P);
    #pragma omp parallel for schedule(static)
    for (int cell = 0; cell < ncell; ++cell) {
        if (s->solid[cell]) continue;
        const moms *m = &K[cell];
        const prim_t *Pn = &P[cell];
        for (int v = 0; v < s->nv; ++v) {
            double xi[3], w;
            node_xi(s, v, xi, &w);
            double Mn = maxwellian(Pn->rho, Pn->u, Pn->Tt, xi);
            double Mo = maxwellian(m->rho, m->u, m->Tt, xi);
            size_t at = (size_t)cell * s->nv + v;
            s->f0[at] += Mn - Mo;
            if (dia) s->f1[at] += 0.5 * c->dr * (Pn->Tr * Mn - m->Tr * Mo);
        }
    }
    free(K); free(Fkin); free(Fint); free(P);
    return s->status;
}

int orc_gsis_correct(orc_state *s, int iters) { return gsis_correct_mode(s, iters, 0); }

/* Initial field of Alg. 1, line 1: macro_steps iterations of the macroscopic
 * solver with the Euler constitutive relations from the current state, the
 * VDF corrected to the result (Eq. updatef), then kinetic_steps passes. */
int orc_gsis_precondition(orc_state *s, int macro_steps, int kinetic_steps)
{
    int st = gsis_correct_mode(s, macro_steps, 1);
    if (st) return st;
    orc_step(s, kinetic_steps);
    return s->status;
}

/* W^{n+1} = (rho, rho u, E, Er) of the last macroscopic solve, out[ncell][6]
 * (zeros in solid cells); returns -1 before any solve. */
int orc_last_macro_W(const orc_state *s, double *out)
{
    if (!s->lastW) return -1;
    for (int cell = 0; cell < s->ncell; ++cell)
        for (int k = 0; k < 6; ++k) out[(size_t)cell * 6 + k] = s->solid[cell] ? 0.0 : s->lastW[(size_t)cell * 6 + k];
    return 0;
}

/* The Navier-Stokes-Fourier closure of the macroscopic solve at the face
 * between fluid cell `cell` and its +a neighbour, for the conservative field
 * W[ncell][6] (rho, rho u, E, Er): out = (sigma_xa, sigma_ya, sigma_za, q_a,
 * qr_a), exactly as the face flux of the iteration evaluates it (no HoT).
 * Returns -1 if that neighbour is not a fluid cell. */
int orc_nsf_face(const orc_state *s, const double *W, int cell, int a, double out[5])
{
    if (s->umesh) return -2;
    if (cell < 0 || cell >= s->ncell || a < 0 || a > 2 || s->solid[cell]) return -1;
    int nb = neighbour(s, cell, 2 * a + 1);
    if (nb < 0) return -1;
    macpar mp;
    macro_params(s, &mp);
    mp.euler = 0;
    prim_t *P = calloc((size_t)s->ncell, sizeof(prim_t));
    for (int c = 0; c < s->ncell; ++c)
        if (!s->solid[c]) prim_of(&mp, W + (size_t)c * 6, &P[c]);
    double gL[9], gR[9], sig[3], q, qr;
    cell_grad(s, P, cell, gL);
    cell_grad(s, P, nb, gR);
    nsf_face(&mp, &P[cell], &P[nb], gL, gR, a, s->h[a], sig, &q, &qr);
    for (int b = 0; b < 3; ++b) out[b] = sig[b];
    out[3] = q;
    out[4] = qr;
    free(P);
    return 0;
}

/* The Grad-13 distributions of Eq. (G13_VDF) (g13_vdf) of the state (rho, u,
 * Tt, Tr) with sq = (sigma xx yy zz xy xz yz, q, qr), at n velocities
 * xi[n][3]: f0[n], f1[n] (f1 zero for the monatomic gas of c). */
void orc_g13_vdf(const orc_cfg *c, double rho, const double u[3], double Tt, double Tr, const double sq[12], int n,
                 const double *xi, double *f0, double *f1)
{
    prim_t P;
    memset(&P, 0, sizeof P);
    P.rho = rho;
    for (int a = 0; a < 3; ++a) P.u[a] = u[a];
    P.Tt = Tt;
    P.Tr = Tr;
    double pre = pow(M_PI * Tt, -1.5);
    for (int i = 0; i < n; ++i) g13_vdf(c, &P, pre, sq, xi + 3 * i, &f0[i], &f1[i]);
}

/* The model flux out of boundary face d (0..5 = -x, +x, -y, +y, -z, +z) of a
 * fluid cell whose W = (rho, rho u, E, Er) is W6, with the boundary rule of
 * that face (model_face_flux): the Maxwellian's with sq == NULL, else the
 * Grad-13 distributions' of sq (as orc_g13_vdf).  Returns -1 if the face is
 * not a boundary face of a fluid cell. */
int orc_model_face_flux(const orc_state *s, const double W6[6], const double *sq, int cell, int d, double F[6])
{
    if (s->umesh || cell < 0 || cell >= s->ncell || d < 0 || d > 5 || s->solid[cell]) return -1;
    int n = neighbour(s, cell, d);
    if (n >= 0) return -1;
    macpar mp;
    macro_params(s, &mp);
    prim_t P;
    prim_of(&mp, W6, &P);
    model_face_flux(s, &P, sq, d, -1 - n, F);
    return 0;
}

/* The stress and heat fluxes the Grad-13 wall flux takes at fluid cell `cell`
 * for the iterate Wm[ncell][6] (rho, rho u, E, Er), the current VDF standing
 * for f^{n+1/2}: NSF_c(W^m) + HoT_c with HoT_c = kinetic - NSF_c(W^{n+1/2}),
 * W^{n+1/2} from the moments of the VDF (g13_cell_hot, g13_cell_stress).
 * sq[12] as orc_g13_vdf.  Returns -1 for a solid or out-of-range cell. */
int orc_g13_wall_stress(const orc_state *s, const double *Wm, int cell, double sq[12])
{
    if ((s->umesh && !s->ucen) || cell < 0 || cell >= s->ncell || s->solid[cell]) return -1;
    const orc_cfg *c = &s->c;
    macpar mp;
    macro_params(s, &mp);
    int ncell = s->ncell;
    moms K;
    prim_t *P = calloc((size_t)ncell, sizeof(prim_t));
    double W[6];
    for (int i = 0; i < ncell; ++i) {
        if (s->solid[i]) continue;
        moms m;
        cell_moments(s, i, &m);
        if (i == cell) K = m;
        double u2 = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
        double Er = mp.dia ? 0.5 * c->dr * m.rho * m.Tr : 0.0;
        W[0] = m.rho;
        for (int a = 0; a < 3; ++a) W[1 + a] = m.rho * m.u[a];
        W[4] = m.rho * u2 + 1.5 * m.rho * m.Tt + Er;
        W[5] = Er;
        prim_of(&mp, W, &P[i]);
    }
    double hot[12];
    g13_cell_hot(s, &mp, &K, P, cell, hot);
    for (int i = 0; i < ncell; ++i)
        if (!s->solid[i]) prim_of(&mp, Wm + (size_t)i * 6, &P[i]);
    g13_cell_stress(s, &mp, P, cell, hot, sq);
    free(P);
    return 0;
}

/* Total mass sum rho V of the current VDF (closed-cavity drift diagnostic). */
/* The least-squares velocity gradients of the unstructured macroscopic solve
 * for a field W[ncell][6]: G[ncell][9], G[b*3+c] = d u_b / d x_c; -2 without
 * an unstructured mesh with centroids. */
int orc_umesh_grad(const orc_state *s, const double *W, double *G)
{
    if (!s->umesh || !s->ucen) return -2;
    macpar mp;
    macro_params(s, &mp);
    prim_t *P = calloc((size_t)s->ncell, sizeof(prim_t));
    for (int i = 0; i < s->ncell; ++i) prim_of(&mp, W + (size_t)i * 6, &P[i]);
    for (int i = 0; i < s->ncell; ++i) ucell_grad(s, P, i, G + (size_t)i * 9);
    free(P);
    return 0;
}

double orc_total_mass(const orc_state *s)
{
    nsum m = {0, 0};
    for (int cell = 0; cell < s->ncell; ++cell) {
        if (s->solid[cell]) continue;
        const double *f0 = s->f0 + (size_t)cell * s->nv;
        nsum r = {0, 0};
        for (int v = 0; v < s->nv; ++v) {
            double xi[3], w;
            node_xi(s, v, xi, &w);
            nadd(&r, w * f0[v]);
        }
        nadd(&m, nval(&r) * (s->umesh ? s->uvol[cell] : 1.0));
    }
    return nval(&m) * (s->umesh ? 1.0 : s->h[0] * s->h[1] * s->h[2]);
}

/* Heat-conduction coefficients k_t, k_r of the macroscopic solve, with
 * q = -(k Tt^omega / delta) grad T in the units above (Eq. (mu_kappa)). */
void orc_conductivities(const orc_cfg *c, double out[2])
{
    orc_state s;
    memset(&s, 0, sizeof s);
    s.c = *c;
    s.delta = 1.0;
    macpar mp;
    macro_params(&s, &mp);
    out[0] = mp.kt;
    out[1] = mp.kr;
}

/* ----------------------------------------------------------- streaming -- */
/* The same iteration for problems whose VDF does not fit in host memory
 * (source iteration 1/dt = 0, first-order fluxes).  A pass needs of f^n only
 * the per-cell moments (the reference distribution) and the outgoing
 * half-range mass flux of each wall face (the wall density), and Eq.
 * (updatef) adds a Maxwellian difference whose sums can be formed directly:
 * so the VDF is never stored.  Each velocity node is swept over all cells as
 * in one_pass, and its values are added to per-cell sums of
 *   w (1, c, c c, c |c|^2) f0  and  w (1, c) f1,   c = xi - u_r,
 * taken about the cell's velocity u_r at the start of the pass (so that the
 * central moments come out without large cancellation), and to per-face sums
 * of the outgoing flux w xi_n (1, xi, |xi|^2 f0 + f1, f1).  This is the
 * stored-VDF path's arithmetic in another loop order (pinned to it on small
 * problems). */
#define ST_NS 17   /* per-cell sums: 1, c (3), cc (xx yy zz xy xz yz), c|c|^2 (3); f1: 1, c (3) */
#define ST_NH 36   /* per-cell half-range fluxes: 3 axes x 2 halves x psi (1, xi, |xi|^2 f0 + f1, f1) */

typedef struct {
    orc_state *s;
    int nface;
    int *fcell, *fdir, *fbc;   /* boundary faces of fluid cells */
    int *cface;                /* [ncell][6] face index, or -1 for an interior face */
    double *ur;                /* [ncell][3] centre of the per-cell sums */
    nsum *acc;                 /* [ncell][ST_NS] */
    nsum *half;                /* [ncell][3][2][6] per axis a: sum over xi_a > 0 (then xi_a < 0) of w xi_a psi f */
    nsum *fout;                /* [nface][6] */
    double in_mass[6][ORC_NBC];    /* sum_{xi_n < 0} w |xi_n| M(1, u_b, T_b) per face direction and slot */
    double in_flux[6][ORC_NBC][6]; /* sum_{xi_n < 0} w xi_n psi M(1, u_b, T_b) (f1 part: (dr/2) T_b M) */
} orc_stream;

void orc_stream_free(orc_stream *st)
{
    if (!st) return;
    orc_free(st->s);
    free(st->fcell); free(st->fdir); free(st->fbc); free(st->cface);
    free(st->ur); free(st->acc); free(st->half); free(st->fout);
    free(st);
}

orc_stream *orc_stream_create(const orc_cfg *cfg, const unsigned char *solid)
{
    if (cfg->inv_dt != 0.0 || cfg->order != 1 || cfg->ucells > 0) return NULL;
    orc_stream *st = calloc(1, sizeof(*st));
    st->s = create_state(cfg, solid, 0);
    if (!st->s) { free(st); return NULL; }
    orc_state *s = st->s;
    const orc_cfg *c = &s->c;
    int ncell = s->ncell;
    st->cface = malloc(sizeof(int) * (size_t)ncell * 6);
    int nf = 0;
    for (int cell = 0; cell < ncell; ++cell)
        for (int d = 0; d < 6; ++d) {
            int n = s->solid[cell] ? 0 : neighbour(s, cell, d);
            st->cface[cell * 6 + d] = n < 0 ? nf++ : -1;
        }
    st->nface = nf;
    st->fcell = malloc(sizeof(int) * (size_t)(nf + 1));
    st->fdir = malloc(sizeof(int) * (size_t)(nf + 1));
    st->fbc = malloc(sizeof(int) * (size_t)(nf + 1));
    for (int cell = 0; cell < ncell; ++cell)
        for (int d = 0; d < 6; ++d) {
            int f = st->cface[cell * 6 + d];
            if (f < 0) continue;
            st->fcell[f] = cell;
            st->fdir[f] = d;
            st->fbc[f] = -1 - neighbour(s, cell, d);
        }
    st->ur = calloc((size_t)ncell * 3, sizeof(double));
    st->acc = calloc((size_t)ncell * ST_NS, sizeof(nsum));
    st->half = calloc((size_t)ncell * ST_NH, sizeof(nsum));
    st->fout = calloc((size_t)(nf + 1) * 6, sizeof(nsum));
    /* the incoming halves of the boundary Maxwellians, once per direction and slot */
    for (int d = 0; d < 6; ++d)
        for (int b = 0; b < ORC_NBC; ++b) {
            int a = d / 2;
            double sg = (d & 1) ? 1.0 : -1.0;
            nsum in = {0, 0}, fl[6];
            memset(fl, 0, sizeof fl);
            for (int v = 0; v < s->nv; ++v) {
                double xi[3], w;
                node_xi(s, v, xi, &w);
                double xn = sg * xi[a];
                if (!(xn < 0)) continue;
                double M = maxwellian(1.0, c->bc_u[b], c->bc_T[b], xi);
                double M1 = c->species == 1 ? 0.5 * c->dr * c->bc_T[b] * M : 0.0;
                double x2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
                double ww = w * xn;
                nadd(&in, w * (-xn) * M);
                nadd(&fl[0], ww * M);
                for (int k = 0; k < 3; ++k) nadd(&fl[1 + k], ww * xi[k] * M);
                nadd(&fl[4], ww * (x2 * M + M1));
                nadd(&fl[5], ww * M1);
            }
            st->in_mass[d][b] = nval(&in);
            for (int k = 0; k < 6; ++k) st->in_flux[d][b][k] = nval(&fl[k]);
        }
    return st;
}

/* Adds the contribution of value f0 (f1) at node xi, weight w, to the sums of
 * one cell (centre ur), its half-range fluxes H and its outgoing boundary
 * faces. */
static void stream_add(const orc_stream *st, nsum *A, nsum *H, nsum *F, const int *cf, const double ur[3],
                       const double xi[3], double w, double f0, double f1, int dia)
{
    double cp[3] = {xi[0] - ur[0], xi[1] - ur[1], xi[2] - ur[2]};
    double c2 = cp[0] * cp[0] + cp[1] * cp[1] + cp[2] * cp[2];
    double wf = w * f0;
    nadd(&A[0], wf);
    for (int a = 0; a < 3; ++a) nadd(&A[1 + a], wf * cp[a]);
    nadd(&A[4], wf * cp[0] * cp[0]);
    nadd(&A[5], wf * cp[1] * cp[1]);
    nadd(&A[6], wf * cp[2] * cp[2]);
    nadd(&A[7], wf * cp[0] * cp[1]);
    nadd(&A[8], wf * cp[0] * cp[2]);
    nadd(&A[9], wf * cp[1] * cp[2]);
    for (int a = 0; a < 3; ++a) nadd(&A[10 + a], wf * cp[a] * c2);
    if (dia) {
        double w1 = w * f1;
        nadd(&A[13], w1);
        for (int a = 0; a < 3; ++a) nadd(&A[14 + a], w1 * cp[a]);
    }
    double x2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
    for (int a = 0; a < 3; ++a) {
        if (xi[a] == 0.0) continue;
        nsum *h = H + a * 12 + (xi[a] > 0 ? 0 : 6);
        double ww = w * xi[a];
        double g1 = dia ? f1 : 0.0;
        nadd(&h[0], ww * f0);
        for (int k = 0; k < 3; ++k) nadd(&h[1 + k], ww * xi[k] * f0);
        nadd(&h[4], ww * (x2 * f0 + g1));
        nadd(&h[5], ww * g1);
    }
    for (int d = 0; d < 6; ++d) {
        int f = cf[d];
        if (f < 0) continue;
        double xn = ((d & 1) ? 1.0 : -1.0) * xi[d / 2];
        if (!(xn > 0)) continue;
        nsum *o = F + (size_t)f * 6;
        double ww = w * xn;
        double g1 = dia ? f1 : 0.0;
        nadd(&o[0], ww * f0);
        for (int k = 0; k < 3; ++k) nadd(&o[1 + k], ww * xi[k] * f0);
        nadd(&o[4], ww * (x2 * f0 + g1));
        nadd(&o[5], ww * g1);
    }
    (void)st;
}

/* Eq. (getmoment) from the sums of a cell: with d = u - u_r = S1 / rho,
 * sum w c c f = S2 - rho d d and sum w c |c|^2 f = S3 - 2 S2 d - d tr S2 + 2 rho |d|^2 d. */
static void stream_moments(const orc_stream *st, int cell, moms *m)
{
    const nsum *A = st->acc + (size_t)cell * ST_NS;
    const double *ur = st->ur + (size_t)cell * 3;
    double S[ST_NS];
    for (int k = 0; k < ST_NS; ++k) S[k] = nval(&A[k]);
    double rho = S[0], d[3];
    for (int a = 0; a < 3; ++a) d[a] = S[1 + a] / rho;
    m->rho = rho;
    for (int a = 0; a < 3; ++a) m->u[a] = ur[a] + d[a];
    double M2[3][3] = {{S[4], S[7], S[8]}, {S[7], S[5], S[9]}, {S[8], S[9], S[6]}};
    double C[6] = {S[4] - rho * d[0] * d[0], S[5] - rho * d[1] * d[1], S[6] - rho * d[2] * d[2],
                   S[7] - rho * d[0] * d[1], S[8] - rho * d[0] * d[2], S[9] - rho * d[1] * d[2]};
    double tr = C[0] + C[1] + C[2];
    m->Tt = (2.0 / 3.0) * tr / rho;
    for (int k = 0; k < 6; ++k) m->sig[k] = 2.0 * (C[k] - (k < 3 ? tr / 3.0 : 0.0));
    double trS = S[4] + S[5] + S[6], dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    for (int a = 0; a < 3; ++a) {
        double Md = M2[a][0] * d[0] + M2[a][1] * d[1] + M2[a][2] * d[2];
        m->q[a] = S[10 + a] - 2.0 * Md - d[a] * trS + 2.0 * rho * dd * d[a];
    }
    if (st->s->c.species == 1) {
        double dr = st->s->c.dr;
        m->Tr = 2.0 * S[13] / (dr * rho);
        for (int a = 0; a < 3; ++a) m->qr[a] = S[14 + a] - d[a] * S[13];
        m->T = (3.0 * m->Tt + dr * m->Tr) / (3.0 + dr);
    } else {
        m->Tr = m->Tt;
        m->qr[0] = m->qr[1] = m->qr[2] = 0.0;
        m->T = m->Tt;
    }
}

static void stream_snapshot(orc_stream *st)
{
    orc_state *s = st->s;
    for (int cell = 0; cell < s->ncell; ++cell) {
        double *pv = s->prev + (size_t)cell * 5;
        if (s->solid[cell]) { memset(pv, 0, 5 * sizeof(double)); continue; }
        moms m;
        stream_moments(st, cell, &m);
        pv[0] = m.rho; pv[1] = m.u[0]; pv[2] = m.u[1]; pv[3] = m.u[2]; pv[4] = m.Tt;
    }
}

/* f0 = M(rho, u, T), f1 = (dr/2) Tr f0 in every fluid cell: the same values
 * in every cell, so their sums are formed once (about u) and copied. */
void orc_stream_init_maxwellian(orc_stream *st, double rho, const double u[3], double T, double Tr)
{
    orc_state *s = st->s;
    int dia = s->c.species == 1;
    nsum A[ST_NS], H[ST_NH], F[6 * 6];
    memset(A, 0, sizeof A);
    memset(H, 0, sizeof H);
    memset(F, 0, sizeof F);
    int cf[6] = {0, 1, 2, 3, 4, 5};   /* all six directions, one sum each */
    for (int v = 0; v < s->nv; ++v) {
        double xi[3], w;
        node_xi(s, v, xi, &w);
        double f0 = maxwellian(rho, u, T, xi);
        double f1 = dia ? 0.5 * s->c.dr * Tr * f0 : 0.0;
        stream_add(st, A, H, F, cf, u, xi, w, f0, f1, dia);
    }
    memset(st->fout, 0, sizeof(nsum) * (size_t)(st->nface + 1) * 6);
    for (int cell = 0; cell < s->ncell; ++cell) {
        for (int a = 0; a < 3; ++a) st->ur[cell * 3 + a] = u[a];
        nsum *dst = st->acc + (size_t)cell * ST_NS, *hd = st->half + (size_t)cell * ST_NH;
        if (s->solid[cell]) {
            memset(dst, 0, sizeof(nsum) * ST_NS);
            memset(hd, 0, sizeof(nsum) * ST_NH);
            continue;
        }
        memcpy(dst, A, sizeof A);
        memcpy(hd, H, sizeof H);
    }
    for (int f = 0; f < st->nface; ++f) memcpy(st->fout + (size_t)f * 6, F + (size_t)st->fdir[f] * 6, 6 * sizeof(nsum));
    s->status = 0;
    stream_snapshot(st);
}

int orc_stream_step(orc_stream *st, int npasses)
{
    orc_state *s = st->s;
    const orc_cfg *c = &s->c;
    int ncell = s->ncell, nv = s->nv, dia = c->species == 1, nf = st->nface;
    cellpar *P = malloc(sizeof(cellpar) * (size_t)ncell);
    double *scale = calloc((size_t)ncell * 6, sizeof(double));
    int *nb = malloc(sizeof(int) * (size_t)ncell * 6);
    for (int pass = 0; pass < npasses; ++pass) {
        #pragma omp parallel for schedule(dynamic, 16)
        for (int cell = 0; cell < ncell; ++cell) {
            if (s->solid[cell]) continue;
            moms m;
            stream_moments(st, cell, &m);
            params_from_moments(s, &m, &P[cell]);
            for (int d = 0; d < 6; ++d) {
                int n = neighbour(s, cell, d);
                nb[cell * 6 + d] = n;
                if (n >= 0) { scale[cell * 6 + d] = 0.0; continue; }
                int bc = -1 - n, f = st->cface[cell * 6 + d];
                scale[cell * 6 + d] = c->bc_kind[bc] == ORC_INFLOW ? c->bc_rho[bc]
                                      : nval(&st->fout[(size_t)f * 6]) / st->in_mass[d][bc];
            }
        }
        for (int cell = 0; cell < ncell; ++cell) {
            if (s->solid[cell]) continue;
            if (!isfinite(P[cell].invtau) || !(P[cell].m.rho > 0) || !(P[cell].m.Tt > 0)) s->status = -5;
            for (int a = 0; a < 3; ++a) st->ur[cell * 3 + a] = P[cell].m.u[a];
        }
        memset(st->acc, 0, sizeof(nsum) * (size_t)ncell * ST_NS);
        memset(st->half, 0, sizeof(nsum) * (size_t)ncell * ST_NH);
        memset(st->fout, 0, sizeof(nsum) * (size_t)(nf + 1) * 6);
        #pragma omp parallel
        {
            double *col0 = calloc((size_t)ncell, sizeof(double));
            double *col1 = calloc((size_t)ncell, sizeof(double));
            nsum *A = calloc((size_t)ncell * ST_NS, sizeof(nsum));
            nsum *Hh = calloc((size_t)ncell * ST_NH, sizeof(nsum));
            nsum *F = calloc((size_t)(nf + 1) * 6, sizeof(nsum));
            /* f^n enters the update only times 1/dt = 0: the columns keep the
             * previous node's (finite) values, or zeros */
            #pragma omp for schedule(static)
            for (int v = 0; v < nv; ++v) {
                double xi[3], w;
                node_xi(s, v, xi, &w);
                sweep_node(s, v, P, scale, nb, col0, col1);
                for (int cell = 0; cell < ncell; ++cell) {
                    if (s->solid[cell]) continue;
                    stream_add(st, A + (size_t)cell * ST_NS, Hh + (size_t)cell * ST_NH, F, st->cface + (size_t)cell * 6,
                               st->ur + (size_t)cell * 3, xi, w, col0[cell], col1[cell], dia);
                }
            }
            /* combine the threads' sums in thread order */
            #pragma omp for ordered schedule(static, 1)
            for (int t = 0; t < omp_get_num_threads(); ++t) {
                #pragma omp ordered
                {
                    for (size_t k = 0; k < (size_t)ncell * ST_NS; ++k) { nadd(&st->acc[k], A[k].s); nadd(&st->acc[k], A[k].c); }
                    for (size_t k = 0; k < (size_t)ncell * ST_NH; ++k) { nadd(&st->half[k], Hh[k].s); nadd(&st->half[k], Hh[k].c); }
                    for (size_t k = 0; k < (size_t)nf * 6; ++k) { nadd(&st->fout[k], F[k].s); nadd(&st->fout[k], F[k].c); }
                }
            }
            free(col0); free(col1); free(A); free(Hh); free(F);
        }
    }
    free(P); free(scale); free(nb);
    return s->status;
}

/* gsis_correct without the VDF: the kinetic boundary flux of each face is its
 * outgoing sums plus the incoming boundary values (wall density recomputed
 * from the outgoing mass flux of f^{n+1/2}), the macroscopic solve as on the
 * stored VDF, and Eq. (updatef) added to the sums node by node. */
int orc_stream_gsis_correct(orc_stream *st, int iters)
{
    orc_state *s = st->s;
    const orc_cfg *c = &s->c;
    int ncell = s->ncell, dia = c->species == 1;
    moms *K = calloc((size_t)ncell, sizeof(moms));
    double *Fkin = calloc((size_t)ncell * 36, sizeof(double));
    double *Fint = calloc((size_t)ncell * 18, sizeof(double));
    prim_t *P = calloc((size_t)ncell, sizeof(prim_t));
    for (int cell = 0; cell < ncell; ++cell) {
        if (s->solid[cell]) continue;
        stream_moments(st, cell, &K[cell]);
        for (int a = 0; a < 3; ++a) {
            /* interior face to the +a neighbour: this cell's xi_a > 0 half plus
             * the neighbour's xi_a < 0 half */
            int n = neighbour(s, cell, 2 * a + 1);
            if (n < 0) continue;
            const nsum *hp = st->half + (size_t)cell * ST_NH + a * 12, *hm = st->half + (size_t)n * ST_NH + a * 12 + 6;
            for (int k = 0; k < 6; ++k) Fint[(size_t)cell * 18 + a * 6 + k] = nval(&hp[k]) + nval(&hm[k]);
        }
        for (int d = 0; d < 6; ++d) {
            int f = st->cface[cell * 6 + d];
            if (f < 0) continue;
            int bc = st->fbc[f];
            const nsum *o = st->fout + (size_t)f * 6;
            double sc = c->bc_kind[bc] == ORC_INFLOW ? c->bc_rho[bc] : nval(&o[0]) / st->in_mass[d][bc];
            double *F = Fkin + (size_t)cell * 36 + d * 6;
            for (int k = 0; k < 6; ++k) F[k] = nval(&o[k]) + sc * st->in_flux[d][bc][k];
            if (!dia) F[5] = 0.0;
        }
    }
    macro_solve(s, K, Fkin, Fint, iters, 0, P);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int cell = 0; cell < ncell; ++cell) {
        if (s->solid[cell]) continue;
        const moms *m = &K[cell];
        const prim_t *Pn = &P[cell];
        double pn = pow(M_PI * Pn->Tt, -1.5), po = pow(M_PI * m->Tt, -1.5);
        nsum *A = st->acc + (size_t)cell * ST_NS;
        for (int v = 0; v < s->nv; ++v) {
            double xi[3], w;
            node_xi(s, v, xi, &w);
            double Mn = maxwellian_pre(Pn->rho, pn, Pn->u, Pn->Tt, xi);
            double Mo = maxwellian_pre(m->rho, po, m->u, m->Tt, xi);
            double d0 = Mn - Mo;
            double d1 = dia ? 0.5 * c->dr * (Pn->Tr * Mn - m->Tr * Mo) : 0.0;
            stream_add(st, A, st->half + (size_t)cell * ST_NH, st->fout, st->cface + (size_t)cell * 6,
                       st->ur + (size_t)cell * 3, xi, w, d0, d1, dia);
        }
    }
    free(K); free(Fkin); free(Fint); free(P);
    return s->status;
}

/* out[ncell][14 or 18] as orc_moments; NaN in solid cells. */
void orc_stream_moments(const orc_stream *st, double *out)
{
    const orc_state *s = st->s;
    int nm = s->c.species == 1 ? 18 : 14;
    for (int cell = 0; cell < s->ncell; ++cell) {
        double *o = out + (size_t)cell * nm;
        if (s->solid[cell]) { for (int k = 0; k < nm; ++k) o[k] = NAN; continue; }
        moms m;
        stream_moments(st, cell, &m);
        o[0] = m.rho; o[1] = m.u[0]; o[2] = m.u[1]; o[3] = m.u[2]; o[4] = m.Tt;
        for (int k = 0; k < 6; ++k) o[5 + k] = m.sig[k];
        for (int a = 0; a < 3; ++a) o[11 + a] = m.q[a];
        if (nm == 18) { o[14] = m.Tr; for (int a = 0; a < 3; ++a) o[15 + a] = m.qr[a]; }
    }
}

/* Eq. (convergence_critertion) as orc_residual, from the sums. */
void orc_stream_residual(orc_stream *st, double eps[3])
{
    orc_state *s = st->s;
    nsum num[3], den[3];
    memset(num, 0, sizeof num); memset(den, 0, sizeof den);
    for (int cell = 0; cell < s->ncell; ++cell) {
        if (s->solid[cell]) continue;
        moms m;
        stream_moments(st, cell, &m);
        const double *pv = s->prev + (size_t)cell * 5;
        double dr = m.rho - pv[0], dT = m.Tt - pv[4];
        nadd(&num[0], dr * dr); nadd(&den[0], pv[0] * pv[0]);
        for (int a = 0; a < 3; ++a) { double du = m.u[a] - pv[1 + a]; nadd(&num[1], du * du); nadd(&den[1], pv[1 + a] * pv[1 + a]); }
        nadd(&num[2], dT * dT); nadd(&den[2], pv[4] * pv[4]);
    }
    double ufloor = (1e3 * 2.220446049250313e-16) * (1e3 * 2.220446049250313e-16) * nval(&den[2]);
    for (int k = 0; k < 3; ++k) {
        double n = nval(&num[k]), d = nval(&den[k]);
        eps[k] = d > (k == 1 ? ufloor : 0.0) ? sqrt(n / d) : sqrt(n);
    }
    stream_snapshot(st);
}

int orc_stream_status(const orc_stream *st) { return st->s->status; }

// libgsis host runtime: argument checks, geometry metadata, workspace
// carving and the kernel sequence behind every C-ABI entry point.
#include "gsis.h"
#include "gsis_common.h"
#include "gsis_launch.h"
#include "gsis_resid_host.h"

#include <algorithm>
#include <map>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace gsis;

struct gsis_ctx {
    gsis_config cfg;
    Geo g;
    BcInfo bc;
    bool fp32 = false;
    std::vector<uint8_t> mask;
    bool meta_ready = false;
    std::vector<int> cflag, nbr, face_cell, face_dir, face_bc, perm;
    std::vector<double> xi[3], w[3];
    std::vector<double> vlist;   // node list [nv][4] in the caller's order (list mode)
    // unstructured spatial mesh (g.umesh): what the sweep needs, built when the
    // mesh is set (see Dev for the meaning of each array)
    std::vector<double> uvol, ucf_g, ubf_n, ucf_lsq, uf_geo;
    std::vector<int> ucf_nb, ucf_meta, ulev, ulev_off, ubf_cell, ubf_slot, uperm, ucls;   // ulev: 2 ints per entry
    std::vector<int> ucf_face, uf_cell, ucf_first, ubf_face;
    int tx = 0, ty = 0, tz = 0, bs = 0;
    std::vector<int> tiles, plane_off, plane_cnt, npblk;
    std::vector<int> tent, nclean;   // split sweep entries (cases with solid cells)
    int vw = 1;
    Dev d;
    Case hcase;              // host copy of the device-resident case record
    Case *dcase = nullptr;   // in the workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool bound = false, inited = false, pending = false, stepped = false;
    long long passes = 0;
    hipStream_t stream = nullptr;
    DivWatch watch;          // divergence reference of the residual
    std::string err;
    // phase timing
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_open;
    double prof_ms[GSIS_NPHASE] = {0};
    long long prof_calls[GSIS_NPHASE] = {0};
    ~gsis_ctx()
    {
        for (auto &e : ev_open) { (void)hipEventDestroy(e.second.first); (void)hipEventDestroy(e.second.second); }
        for (auto e : ev_pool) hipEventDestroy(e);
    }
};

namespace {

gsis_status fail(gsis_ctx *c, gsis_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

#define HIPCHK(ctx, expr)                                                                              \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return fail(ctx, GSIS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool finite3(const double *u) { return u && std::isfinite(u[0]) && std::isfinite(u[1]) && std::isfinite(u[2]); }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <class P> void carve(size_t &off, P *&ptr, size_t count, char *base)
{
    off = align256(off);
    ptr = base ? (P *)(base + off) : nullptr;
    off += count * sizeof(P);
}

void default_tile(gsis_ctx *c)
{
    bool dia = c->g.species == GSIS_DIATOMIC;
    if (c->fp32) { c->tx = 8; c->ty = dia ? 4 : 8; c->tz = 8; c->bs = 128; }
    else { c->tx = 4; c->ty = 4; c->tz = 4; c->bs = 128; }
}

int sweep_nvb(const Geo &g, int bs)
{
    int omax = 0;
    for (int o = 0; o < 8; ++o) omax = std::max(omax, g.osize[o]);
    return (omax + bs - 1) / bs;
}

// velocity nodes per sweep block: one run of 64 for a wave grid (its waves
// share the nodes), the block size otherwise
int block_nodes(const gsis_ctx *c)
{
    return sweep_shape_waves(c->fp32, c->tx, c->ty) > 1 ? 64 : c->bs;
}

// The (tile, octant) entries of every plane for a case with solid cells: an
// entry is clean when no cell of the tile, nor of its upwind halo (one cell
// layer on the inflow side of each axis, in the octant's frame), is solid, so
// the sweep kernel without the solid-cell logic gives the same values there.
// Clean entries come first within each plane.
void build_split(gsis_ctx *c)
{
    const Geo &g = c->g;
    c->tent.clear();
    c->nclean.clear();
    if (g.nfluid == g.ncell || c->cflag.empty()) return;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    // prefix counts of solid cells: P[k][j][i] = solid cells in [0,i) x [0,j) x [0,k)
    const size_t sx = nx + 1, sy = ny + 1;
    std::vector<int> P(sx * sy * (nz + 1), 0);
    auto at = [&](int i, int j, int k) -> int & { return P[(size_t)i + sx * ((size_t)j + sy * k)]; };
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int s = c->cflag[i + nx * (j + ny * k)] ? 0 : 1;
                at(i + 1, j + 1, k + 1) = s + at(i, j + 1, k + 1) + at(i + 1, j, k + 1) + at(i + 1, j + 1, k)
                                          - at(i, j, k + 1) - at(i, j + 1, k) - at(i + 1, j, k) + at(i, j, k);
            }
    auto solid_in = [&](int i0, int i1, int j0, int j1, int k0, int k1) {
        return at(i1, j1, k1) - at(i0, j1, k1) - at(i1, j0, k1) - at(i1, j1, k0) + at(i0, j0, k1) + at(i0, j1, k0)
                   + at(i1, j0, k0) - at(i0, j0, k0) > 0;
    };
    // frame range [lo, hi) along an axis of n cells -> physical range, mirrored for a negative octant half
    auto phys = [](int lo, int hi, int n, bool neg, int &a, int &b) {
        lo = std::max(lo, 0);
        hi = std::min(hi, n);
        a = neg ? n - hi : lo;
        b = neg ? n - lo : hi;
    };
    const int np = (int)c->plane_cnt.size();
    c->nclean.assign(np, 0);
    c->tent.resize(c->tiles.size() * 8);
    for (int p = 0; p < np; ++p) {
        std::vector<int> clean, dirty;
        for (int t = 0; t < c->plane_cnt[p]; ++t) {
            const int pk = c->tiles[c->plane_off[p] + t];
            const int x = pk & 0x3ff, y = (pk >> 10) & 0x3ff, z = (pk >> 20) & 0x3ff;
            for (int o = 0; o < 8; ++o) {
                int a0, a1, b0, b1, d0, d1;
                phys(x * c->tx - 1, (x + 1) * c->tx, nx, o & 1, a0, a1);
                phys(y * c->ty - 1, (y + 1) * c->ty, ny, o & 2, b0, b1);
                phys(z * c->tz - 1, (z + 1) * c->tz, nz, o & 4, d0, d1);
                (solid_in(a0, a1, b0, b1, d0, d1) ? dirty : clean).push_back(t << 3 | o);
            }
        }
        c->nclean[p] = (int)clean.size();
        std::copy(clean.begin(), clean.end(), c->tent.begin() + 8 * (size_t)c->plane_off[p]);
        std::copy(dirty.begin(), dirty.end(), c->tent.begin() + 8 * (size_t)c->plane_off[p] + clean.size());
    }
}

void build_tiles(gsis_ctx *c)
{
    const Geo &g = c->g;
    int ntx = (g.nx + c->tx - 1) / c->tx, nty = (g.ny + c->ty - 1) / c->ty, ntz = (g.nz + c->tz - 1) / c->tz;
    int nplane = ntx + nty + ntz - 2;
    c->tiles.clear();
    c->plane_off.assign(nplane, 0);
    c->plane_cnt.assign(nplane, 0);
    c->npblk.assign(nplane, 0);
    for (int s = 0; s < nplane; ++s) {
        c->plane_off[s] = (int)c->tiles.size();
        for (int z = 0; z < ntz; ++z)
            for (int y = 0; y < nty; ++y) {
                int x = s - y - z;
                if (x < 0 || x >= ntx) continue;
                c->tiles.push_back(x | (y << 10) | (z << 20));
            }
        c->plane_cnt[s] = (int)c->tiles.size() - c->plane_off[s];
        c->npblk[s] = c->plane_cnt[s] * 8 * sweep_nvb(g, block_nodes(c));
    }
    build_split(c);
}

// octant of a node (s_a = 1 when xi_a < 0)
int list_octant(const double *t) { return (t[0] < 0.0 ? 1 : 0) | (t[1] < 0.0 ? 2 : 0) | (t[2] < 0.0 ? 4 : 0); }

// neighbour table, boundary faces, node permutation, moment vector width
void build_meta(gsis_ctx *c)
{
    Geo &g = c->g;
    int nx = g.nx, ny = g.ny, nz = g.nz, n = g.ncell;
    if (g.umesh) {
        // every cell of the mesh is a fluid cell; the box's neighbour table,
        // face list and sweep tiles stay empty
        c->mask.assign(n, 0);
        c->cflag.assign(n, 1);
        c->nbr.assign((size_t)n * 6, -1);
        c->face_cell.clear(); c->face_dir.clear(); c->face_bc.clear();
        g.nface = 0;
        g.nfluid = n;
        c->perm = c->uperm;
        c->vw = 1;
        c->tiles.clear(); c->plane_off.clear(); c->plane_cnt.clear(); c->npblk.clear();
        c->tent.clear(); c->nclean.clear();
        c->meta_ready = true;
        return;
    }
    if (c->mask.empty()) c->mask.assign(n, 0);
    c->cflag.assign(n, 0);
    c->nbr.assign((size_t)n * 6, 0);
    c->face_cell.clear(); c->face_dir.clear(); c->face_bc.clear();
    for (int cell = 0; cell < n; ++cell) c->cflag[cell] = c->mask[cell] ? 0 : 1;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int cell = i + nx * (j + ny * k);
                for (int dir = 0; dir < 6; ++dir) {
                    if (!c->cflag[cell]) { c->nbr[(size_t)cell * 6 + dir] = -1; continue; }
                    int a = dir / 2, sg = (dir & 1) ? 1 : -1;
                    int ii = i + (a == 0 ? sg : 0), jj = j + (a == 1 ? sg : 0), kk = k + (a == 2 ? sg : 0);
                    int bc = -1, nb = -1;
                    if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) bc = dir;
                    else {
                        nb = ii + nx * (jj + ny * kk);
                        if (!c->cflag[nb]) bc = 6;
                    }
                    if (bc >= 0) {
                        int f = (int)c->face_cell.size();
                        c->face_cell.push_back(cell);
                        c->face_dir.push_back(dir);
                        c->face_bc.push_back(bc);
                        c->nbr[(size_t)cell * 6 + dir] = -(f + 1);
                    } else {
                        c->nbr[(size_t)cell * 6 + dir] = nb;
                    }
                }
            }
    g.nface = (int)c->face_cell.size();
    g.nfluid = 0;
    for (int cell = 0; cell < n; ++cell) g.nfluid += c->cflag[cell];
    c->perm.assign(g.nv, 0);
    if (g.vlist) {
        // octant by octant, each in the caller's order
        std::vector<int> at(g.obase, g.obase + 8);
        for (int k = 0; k < g.nv; ++k) c->perm[at[list_octant(&c->vlist[(size_t)k * 4])]++] = k;
    }
    for (int o = 0; o < 8 && !g.vlist; ++o)
        for (int l = 0; l < g.osize[o]; ++l) {
            int nox = g.on[o][0], noy = g.on[o][1];
            int lx = l % nox, r = l / nox, ly = r % noy, lz = r / noy;
            int kx = ((o & 1) ? 0 : g.k0[0]) + lx;
            int ky = ((o & 2) ? 0 : g.k0[1]) + ly;
            int kz = ((o & 4) ? 0 : g.k0[2]) + lz;
            c->perm[g.obase[o] + l] = kx + g.n1[0] * (ky + g.n1[1] * kz);
        }
    int vw = g.vlist ? 1 : (c->fp32 ? 4 : 2);
    while (vw > 1) {
        bool ok = true;
        for (int o = 0; o < 8; ++o)
            if (g.osize[o] > 0 && g.on[o][0] % vw) ok = false;
        if (ok) break;
        vw >>= 1;
    }
    c->vw = vw;
    build_tiles(c);
    c->meta_ready = true;
}

// Layout of the workspace; with base == nullptr only the size is computed.
size_t layout(gsis_ctx *c, char *base)
{
    const Geo &g = c->g;
    Dev &d = c->d;
    size_t off = 0, n = g.ncell, nv = g.nv, esz = c->fp32 ? 4 : 8;
    size_t nf = std::max(g.nface, 1);
    char *f0 = nullptr, *f1 = nullptr;
    carve(off, f0, (n + 1) * nv * esz, base);
    if (g.species == 1) carve(off, f1, (n + 1) * nv * esz, base);
    d.f0 = f0;
    d.f1 = f1;
    d.rs0 = f0;
    d.rs1 = f1;
    d.ho0 = d.ho1 = d.lim0 = d.lim1 = nullptr;
    if (g.order == 2) {
        char *h0 = nullptr, *h1 = nullptr, *l0 = nullptr, *l1 = nullptr;
        carve(off, h0, (n + 1) * nv * esz, base);
        carve(off, l0, n * nv * esz, base);
        if (g.species == 1) {
            carve(off, h1, (n + 1) * nv * esz, base);
            carve(off, l1, n * nv * esz, base);
        }
        d.ho0 = h0; d.ho1 = h1; d.lim0 = l0; d.lim1 = l1;
        d.rs0 = h0; d.rs1 = h1;
    }
    carve(off, d.mom8, n * 8 * NRS, base);
    carve(off, d.cm, n * NMOM, base);
    carve(off, d.par, n * NPAR, base);
    carve(off, d.parf, n * NPAR, base);
    carve(off, d.cflag, n, base);
    carve(off, d.nbr, n * 6, base);
    carve(off, d.face_cell, nf, base);
    carve(off, d.face_dir, nf, base);
    carve(off, d.face_bc, nf, base);
    carve(off, d.fscale, nf, base);
    carve(off, d.fscalef, nf, base);
    carve(off, d.cfs64, n * 6, base);
    carve(off, d.cfs32, n * 6, base);
    d.lsum = nullptr;
    if (g.vlist) carve(off, d.lsum, n * LSUM, base);
    carve(off, d.nt64, nv * 4, base);
    carve(off, d.nt32, nv * 4, base);
    for (int a = 0; a < 3; ++a) {
        carve(off, d.xi64[a], (size_t)g.n1[a], base);
        carve(off, d.xi32[a], (size_t)g.n1[a], base);
        carve(off, d.w64[a], (size_t)g.n1[a], base);
    }
    carve(off, d.xtab, (size_t)g.n1[0] * 4, base);
    carve(off, d.ytab, (size_t)g.n1[1] * 2, base);
    carve(off, d.ztab, (size_t)g.n1[2] * 2, base);
    carve(off, d.mb64, (size_t)NBC * nv, base);
    carve(off, d.mb1_64, (size_t)NBC * nv, base);
    carve(off, d.mb32, (size_t)NBC * nv, base);
    carve(off, d.mb1_32, (size_t)NBC * nv, base);
    carve(off, d.inpsi, (size_t)NBC * 36, base);
    carve(off, d.perm, nv, base);
    carve(off, d.tiles, n, base);
    carve(off, d.plane_off, (size_t)g.nx + g.ny + g.nz, base);
    carve(off, d.tent, 8 * n, base);
    Case *dc = nullptr;
    carve(off, dc, 1, base);
    if (base) c->dcase = dc;
    d.uvol = nullptr; d.ucf_nb = d.ucf_meta = nullptr; d.ucf_g64 = nullptr; d.ucf_g32 = nullptr;
    d.ucls = nullptr; d.ulev = nullptr;
    d.ucf_lsq = nullptr; d.ucf_face = nullptr; d.uf_cell = nullptr; d.ucf_first = nullptr; d.ubf_face = nullptr;
    d.uf_geo = d.uFk = d.ufix = d.uFf = d.ubin = nullptr;
    d.ubsq = d.ubhot = nullptr;
    d.ubf_cell = d.ubf_slot = nullptr; d.ubf_n = nullptr; d.ubf_s64 = nullptr; d.ubf_s32 = nullptr;
    if (g.umesh) {
        const size_t ne = c->ucf_nb.size(), nb = std::max(g.unbf, 1);
        carve(off, d.uvol, n, base);
        carve(off, d.ucf_nb, ne, base);
        carve(off, d.ucf_meta, ne, base);
        carve(off, d.ucf_g64, ne * 4, base);
        carve(off, d.ucf_g32, ne * 4, base);
        carve(off, d.ucls, (size_t)g.ucls, base);
        carve(off, d.ulev, c->ulev.size() / 2, base);
        carve(off, d.ubf_cell, nb, base);
        carve(off, d.ubf_slot, nb, base);
        carve(off, d.ubf_n, nb * 4, base);
        carve(off, d.ubf_s64, nb, base);
        carve(off, d.ubf_s32, nb, base);
        if (g.ucen) {
            const size_t nfc = (size_t)g.unface;
            carve(off, d.ucf_lsq, ne * 3, base);
            carve(off, d.ucf_face, ne, base);
            carve(off, d.ucf_first, n + 1, base);
            carve(off, d.ubf_face, nb, base);
            carve(off, d.uf_cell, nfc * 2, base);
            carve(off, d.uf_geo, nfc * 9, base);
            carve(off, d.uFk, nfc * 6, base);
            carve(off, d.ufix, nfc * 6, base);
            carve(off, d.uFf, nfc * 7, base);
            carve(off, d.ubin, nb * 6, base);
            carve(off, d.ubsq, nb * 12, base);
            carve(off, d.ubhot, nb * 12, base);
        }
    }
    carve(off, d.corr, n * NCORR, base);
    carve(off, d.snap, n * NSNAP, base);
    carve(off, d.W, n * 6, base);
    carve(off, d.W2, n * 6, base);
    carve(off, d.P, n * 12, base);
    carve(off, d.grad, n * 9, base);
    carve(off, d.hot, n * 18, base);
    carve(off, d.R, n * 6, base);
    carve(off, d.Dc, n, base);
    carve(off, d.Src, n, base);
    carve(off, d.fbfix, nf * 6, base);
    carve(off, d.Fb, nf * 6, base);
    carve(off, d.Gb, nf, base);
    carve(off, d.ghot, nf * 12, base);
    carve(off, d.red, (size_t)(resid_blocks(g) + 1) * 6, base);
    carve(off, d.dmax, (size_t)2 * DSLOT * DSTRIDE, base);
    carve(off, d.errflag, 4, base);
    return align256(off);
}

int vw_class(int vw) { return vw >= 4 ? 2 : (vw == 2 ? 1 : 0); }

// The launch target of this context alone.
Target target_of(const gsis_ctx *c)
{
    Target t;
    t.cases = c->dcase;
    t.ncase = 1;
    t.host = &c->hcase;
    for (int k = 0; k < NKIND; ++k) t.nblk[k] = kind_blocks(c->g, (Kind)k);
    t.npblk = c->npblk.data();
    t.nplane = (int)c->npblk.size();
    t.fp32 = c->fp32;
    t.dia = c->g.species == GSIS_DIATOMIC;
    t.mask = c->g.nfluid != c->g.ncell;
    t.rfn = c->g.inv_dt != 0.0 || c->g.order == 2;
    t.mom_nblk[vw_class(c->vw)] = c->g.ncell;
    t.vlist = c->g.vlist != 0;
    t.g13 = c->g.wall_flux == GSIS_WALLFLUX_G13;
    if (!c->nclean.empty()) {
        t.nclean = c->nclean.data();
        t.pcnt = c->plane_cnt.data();
        t.nvb = sweep_nvb(c->g, block_nodes(c));
    }
    t.tx = c->tx;
    t.ty = c->ty;
    t.bs = c->bs;
    return t;
}

// Tile lists, plane offsets and the case record to the device (stream-ordered
// with earlier work: the host waits for the stream first).
hipError_t upload_tiles(gsis_ctx *c)
{
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess && !c->tiles.empty())
        e = hipMemcpy(c->d.tiles, c->tiles.data(), c->tiles.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess && !c->plane_off.empty())
        e = hipMemcpy(c->d.plane_off, c->plane_off.data(), c->plane_off.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess && !c->tent.empty())
        e = hipMemcpy(c->d.tent, c->tent.data(), c->tent.size() * sizeof(int), hipMemcpyHostToDevice);
    c->hcase.g = c->g;
    c->hcase.bc = c->bc;
    c->hcase.d = c->d;
    c->hcase.tz = c->tz;
    c->hcase.nvb = sweep_nvb(c->g, block_nodes(c));
    if (e == hipSuccess) e = hipMemcpy(c->dcase, &c->hcase, sizeof(Case), hipMemcpyHostToDevice);
    return e;
}

gsis_status reset_flags(gsis_ctx *c)
{
    HIPCHK(c, launch_zero_int(c->d.errflag, 4, c->stream));
    return GSIS_OK;
}

// moments of the stored VDF (octant sums, then central moments)
gsis_status reduce_vdf(gsis_ctx *c)
{
    const Target t = target_of(c);
    HIPCHK(c, launch_moments(t, c->stream));
    HIPCHK(c, launch_derive(t, c->stream));
    return GSIS_OK;
}

gsis_status materialize(gsis_ctx *c)
{
    if (!c->pending) return GSIS_OK;
    HIPCHK(c, launch_apply_correction(c->g, c->d, c->fp32, c->stream));
    c->pending = false;
    return GSIS_OK;
}

// Records an event pair around a phase when profiling is on.
struct PhaseTimer {
    gsis_ctx *c;
    int phase;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t take(hipEvent_t &e)
    {
        if (!c->ev_pool.empty()) { e = c->ev_pool.back(); c->ev_pool.pop_back(); return hipSuccess; }
        return hipEventCreate(&e);
    }
    hipError_t start(gsis_ctx *ctx, int ph)
    {
        c = ctx;
        phase = ph;
        if (!c->prof) return hipSuccess;
        hipError_t e = take(a);
        if (e == hipSuccess) e = take(b);
        if (e == hipSuccess) e = hipEventRecord(a, c->stream);
        return e;
    }
    hipError_t stop()
    {
        if (!c->prof || !a) return hipSuccess;
        hipError_t e = hipEventRecord(b, c->stream);
        c->ev_open.push_back({phase, {a, b}});
        return e;
    }
};

struct StateHeader {
    char magic[8];
    int version, ncell, nv, fp32, species, pending, stepped, have_first;   // have_first: bit k = watch.have[k]
    long long passes;
    double first_eps[3];
    char pad[128 - 8 - 9 * 4 - 8 - 24];
};
static_assert(sizeof(StateHeader) == 128, "state header size");

struct StatePart { void *ptr; size_t bytes; };

void state_parts(const gsis_ctx *c, std::vector<StatePart> &parts)
{
    const Geo &g = c->g;
    size_t n = g.ncell, esz = c->fp32 ? 4 : 8;
    parts.clear();
    parts.push_back({c->d.f0, n * g.nv * esz});
    if (g.species == 1) parts.push_back({c->d.f1, n * g.nv * esz});
    parts.push_back({c->d.mom8, n * 8 * NRS * sizeof(double)});
    parts.push_back({c->d.cm, n * NMOM * sizeof(double)});
    parts.push_back({c->d.corr, n * NCORR * sizeof(double)});
    parts.push_back({c->d.snap, n * NSNAP * sizeof(double)});
}

// The rest of a residual once its sums are queued at `total` (device): read
// them and the error flag, take the new snapshot, evaluate eps and the
// divergence watch.  Synchronises.
gsis_status residual_finish(gsis_ctx *ctx, const double *total, PhaseTimer *t, double eps[3])
{
    double sums[6];
    int flag[4];
    HIPCHK(ctx, hipMemcpyAsync(sums, total, sizeof sums, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(flag, ctx->d.errflag, sizeof flag, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, launch_snapshot(target_of(ctx), ctx->stream));
    if (t) HIPCHK(ctx, t->stop());
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    const ResidEval r = resid_eval(sums, ctx->fp32);
    for (int k = 0; k < 3; ++k) eps[k] = r.eps[k];
    if (flag[0] || !std::isfinite(eps[0]) || !std::isfinite(eps[1]) || !std::isfinite(eps[2]))
        return fail(ctx, GSIS_ENOTFINITE, "non-positive or non-finite density/temperature (flag " +
                                              std::to_string(flag[0]) + ")");
    if (resid_diverged(ctx->watch, r, 1e6))
        return fail(ctx, GSIS_EDIVERGED, "residual grew beyond 1e6 times its first relative value");
    return GSIS_OK;
}

}  // namespace

extern "C" {

const char *gsis_last_error(const gsis_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : "no context";
}

// Octant layout of the node set: the first non-negative node per axis (a node
// at 0 belongs to the positive half), octant extents, sizes and bases.
static void octant_layout(gsis_ctx *x)
{
    Geo &g = x->g;
    if (g.vlist) {
        int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int k = 0; k < g.nv; ++k) ++cnt[list_octant(&x->vlist[(size_t)k * 4])];
        int base = 0;
        for (int o = 0; o < 8; ++o) {
            g.on[o][0] = cnt[o];
            g.on[o][1] = g.on[o][2] = 1;
            g.osize[o] = cnt[o];
            g.obase[o] = base;
            base += cnt[o];
        }
        for (int a = 0; a < 3; ++a) g.n1[a] = g.k0[a] = 0;
        return;
    }
    for (int a = 0; a < 3; ++a) {
        const int n = g.n1[a];
        int k0 = n;
        for (int k = 0; k < n; ++k)
            if (k0 == n && x->xi[a][k] >= 0.0) k0 = k;
        g.k0[a] = k0;
    }
    int base = 0;
    for (int o = 0; o < 8; ++o) {
        int sz = 1;
        for (int a = 0; a < 3; ++a) {
            g.on[o][a] = ((o >> a) & 1) ? g.k0[a] : g.n1[a] - g.k0[a];
            sz *= g.on[o][a];
        }
        g.osize[o] = sz;
        g.obase[o] = base;
        base += sz;
    }
}

gsis_status gsis_create(gsis_ctx **out, const gsis_config *cfg)
{
    if (!out) return GSIS_EINVAL;
    *out = nullptr;
    if (!cfg) return GSIS_EINVAL;
    const gsis_config &c = *cfg;
    if (c.nx < 1 || c.ny < 1 || c.nz < 1 || c.nx > 4096 || c.ny > 4096 || c.nz > 4096) return GSIS_EINVAL;
    if (!(c.lx > 0) || !(c.ly > 0) || !(c.lz > 0) || !std::isfinite(c.lx) || !std::isfinite(c.ly) || !std::isfinite(c.lz))
        return GSIS_EINVAL;
    int nvv[3] = {c.nvx, c.nvy, c.nvz};
    for (int a = 0; a < 3; ++a) {
        if (nvv[a] < 2 || nvv[a] > 4096) return GSIS_EINVAL;
        if (!std::isfinite(c.vmin[a]) || !std::isfinite(c.vmax[a]) || !(c.vmax[a] > c.vmin[a])) return GSIS_EINVAL;
    }
    long long nv = (long long)c.nvx * c.nvy * c.nvz;
    long long ncell = (long long)c.nx * c.ny * c.nz;
    if (nv > (1ll << 30) || ncell > (1ll << 30)) return GSIS_EINVAL;
    if (c.species != GSIS_MONATOMIC && c.species != GSIS_DIATOMIC) return GSIS_EINVAL;
    if (!(c.Kn > 0) || !std::isfinite(c.Kn) || !std::isfinite(c.omega)) return GSIS_EINVAL;
    if (c.species == GSIS_DIATOMIC) {
        double det = c.A[0] * c.A[3] - c.A[1] * c.A[2];
        if (!(c.dr > 0) || !(c.Zr >= 1.0) || !std::isfinite(det) || det == 0.0) return GSIS_EINVAL;
    }
    if (!(c.inv_dt >= 0) || !std::isfinite(c.inv_dt)) return GSIS_EINVAL;
    if (c.vdf_dtype != GSIS_FP64 && c.vdf_dtype != GSIS_FP32) return GSIS_EINVAL;
    if (c.conservative != 0 && c.conservative != 1) return GSIS_EINVAL;
    if (!(c.macro_cfl > 0) || !std::isfinite(c.macro_cfl)) return GSIS_EINVAL;
    if (c.order < 0 || c.order > 2 || !std::isfinite(c.limiter_k)) return GSIS_EINVAL;

    gsis_ctx *x = new (std::nothrow) gsis_ctx();
    if (!x) return GSIS_ENOMEM;
    x->cfg = c;
    x->fp32 = c.vdf_dtype == GSIS_FP32;
    Geo &g = x->g;
    std::memset(&g, 0, sizeof g);
    g.nx = c.nx; g.ny = c.ny; g.nz = c.nz;
    g.ncell = (int)ncell;
    g.h[0] = c.lx / c.nx; g.h[1] = c.ly / c.ny; g.h[2] = c.lz / c.nz;
    g.hmin = std::min(g.h[0], std::min(g.h[1], g.h[2]));
    for (int a = 0; a < 3; ++a) {
        g.invh[a] = 1.0 / g.h[a];
        int n = nvv[a];
        g.n1[a] = n;
        double dv = (c.vmax[a] - c.vmin[a]) / (n - 1);
        x->xi[a].resize(n);
        x->w[a].resize(n);
        for (int k = 0; k < n; ++k) {
            x->xi[a][k] = c.vmin[a] + k * dv;
            x->w[a][k] = (k == 0 || k == n - 1) ? 0.5 * dv : dv;
        }
    }
    g.nv = (int)nv;
    octant_layout(x);
    g.species = c.species;
    g.delta = std::sqrt(PI) / (2.0 * c.Kn);
    g.omega = c.omega;
    g.dr = c.species == GSIS_DIATOMIC ? c.dr : 0.0;
    g.Zr = c.species == GSIS_DIATOMIC ? c.Zr : 1.0;
    for (int k = 0; k < 4; ++k) g.A[k] = c.A[k];
    g.inv_dt = c.inv_dt;
    g.order = c.order == 2 ? 2 : 1;
    g.limited = c.limiter_k >= 0;
    {
        const double kh = g.limited ? c.limiter_k * std::cbrt(g.h[0] * g.h[1] * g.h[2]) : 0.0;
        g.venk_e2 = kh * kh * kh;
    }
    g.rs_scale = g.order == 2 ? 1.0 : c.inv_dt;
    g.conservative = c.conservative;
    g.macro_cfl = c.macro_cfl;
    if (c.species == GSIS_DIATOMIC) {
        double det = c.A[0] * c.A[3] - c.A[1] * c.A[2];
        double at = (c.A[3] * 5.0 - c.A[1] * c.dr) / det;
        double ar = (-c.A[2] * 5.0 + c.A[0] * c.dr) / det;
        g.kt = at / 4.0;
        g.kr = ar / 4.0;
        g.gam = (5.0 + c.dr) / (3.0 + c.dr);
    } else {
        g.kt = 15.0 / 8.0;
        g.kr = 0.0;
        g.gam = 5.0 / 3.0;
    }
    double nu = 0.5;
    if (g.kt / 1.5 > nu) nu = g.kt / 1.5;
    if (c.species == GSIS_DIATOMIC && g.kr / (0.5 * c.dr) > nu) nu = g.kr / (0.5 * c.dr);
    g.Cd = 2.0 * nu;
    for (int b = 0; b < NBC; ++b) {
        x->bc.kind[b] = GSIS_DIFFUSE_WALL;
        x->bc.u[b][0] = x->bc.u[b][1] = x->bc.u[b][2] = 0.0;
        x->bc.T[b] = 1.0;
        x->bc.rho[b] = 1.0;
    }
    g.fp32 = x->fp32 ? 1 : 0;
    default_tile(x);
    *out = x;
    return GSIS_OK;
}

gsis_status gsis_destroy(gsis_ctx *ctx)
{
    if (!ctx) return GSIS_EINVAL;
    delete ctx;
    return GSIS_OK;
}

gsis_status gsis_set_velocity_nodes(gsis_ctx *ctx, int axis, const double *nodes, int n)
{
    if (!ctx) return GSIS_EINVAL;
    if (ctx->bound || ctx->meta_ready) return fail(ctx, GSIS_ESTATE, "set_velocity_nodes must precede workspace_size/bind");
    if (axis < 0 || axis > 2) return fail(ctx, GSIS_EINVAL, "axis must be 0, 1 or 2");
    if (ctx->g.vlist) return fail(ctx, GSIS_ESTATE, "the context holds a velocity node list, not a tensor grid");
    if (!nodes) return fail(ctx, GSIS_EINVAL, "nodes is NULL");
    if (n != ctx->g.n1[axis]) return fail(ctx, GSIS_EINVAL, "n must equal the configured node count of the axis");
    for (int k = 0; k < n; ++k)
        if (!std::isfinite(nodes[k]) || (k > 0 && !(nodes[k] > nodes[k - 1])))
            return fail(ctx, GSIS_EINVAL, "nodes must be finite and strictly increasing");
    std::vector<double> &xi = ctx->xi[axis], &w = ctx->w[axis];
    for (int k = 0; k < n; ++k) {
        xi[k] = nodes[k];
        // trapezoid rule on the given nodes: half of each neighbouring gap
        w[k] = 0.5 * ((k < n - 1 ? nodes[k + 1] : nodes[k]) - (k > 0 ? nodes[k - 1] : nodes[k]));
    }
    octant_layout(ctx);
    return GSIS_OK;
}

gsis_status gsis_set_velocity_list(gsis_ctx *ctx, const double *nodes, int n)
{
    if (!ctx) return GSIS_EINVAL;
    if (ctx->bound || ctx->meta_ready) return fail(ctx, GSIS_ESTATE, "set_velocity_list must precede workspace_size/bind");
    if (ctx->g.umesh) return fail(ctx, GSIS_ESTATE, "set_velocity_list must precede set_spatial_mesh");
    if (!nodes) return fail(ctx, GSIS_EINVAL, "nodes is NULL");
    if (n < 2 || n > (1 << 24)) return fail(ctx, GSIS_EINVAL, "the node count must be in [2, 2^24]");
    for (int k = 0; k < n; ++k) {
        const double *t = nodes + (size_t)k * 4;
        if (!std::isfinite(t[0]) || !std::isfinite(t[1]) || !std::isfinite(t[2]))
            return fail(ctx, GSIS_EINVAL, "node velocities must be finite");
        if (!(t[3] > 0.0) || !std::isfinite(t[3])) return fail(ctx, GSIS_EINVAL, "node weights must be positive and finite");
    }
    if ((long long)n * ctx->g.ncell > (1ll << 40)) return fail(ctx, GSIS_EINVAL, "cells x nodes too large");
    ctx->vlist.assign(nodes, nodes + (size_t)n * 4);
    for (int a = 0; a < 3; ++a) { ctx->xi[a].clear(); ctx->w[a].clear(); }
    ctx->g.vlist = 1;
    ctx->g.nv = n;
    octant_layout(ctx);
    return GSIS_OK;
}

// Symmetric 3x3 matrix: its inverse on its range (Jacobi eigen-decomposition,
// eigenvalues below 1e-12 of the largest dropped).
static void sym3_pinv(const double A[9], double Pi[9])
{
    double a[3][3], v[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) a[i][j] = A[i * 3 + j];
    for (int sweep = 0; sweep < 50; ++sweep) {
        if (std::fabs(a[0][1]) + std::fabs(a[0][2]) + std::fabs(a[1][2]) == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (a[p][q] == 0.0) continue;
                const double th = 0.5 * (a[q][q] - a[p][p]) / a[p][q];
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < 3; ++k) {
                    const double x = a[k][p], y = a[k][q];
                    a[k][p] = cs * x - sn * y;
                    a[k][q] = sn * x + cs * y;
                }
                for (int k = 0; k < 3; ++k) {
                    const double x = a[p][k], y = a[q][k];
                    a[p][k] = cs * x - sn * y;
                    a[q][k] = sn * x + cs * y;
                }
                for (int k = 0; k < 3; ++k) {
                    const double x = v[k][p], y = v[k][q];
                    v[k][p] = cs * x - sn * y;
                    v[k][q] = sn * x + cs * y;
                }
            }
    }
    const double emax = std::max(std::fabs(a[0][0]), std::max(std::fabs(a[1][1]), std::fabs(a[2][2])));
    double inv[3];
    for (int k = 0; k < 3; ++k) inv[k] = (emax > 0 && a[k][k] > 1e-12 * emax) ? 1.0 / a[k][k] : 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Pi[i * 3 + j] = v[i][0] * inv[0] * v[j][0] + v[i][1] * inv[1] * v[j][1] + v[i][2] * inv[2] * v[j][2];
}

gsis_status gsis_set_spatial_mesh(gsis_ctx *ctx, int ncell, const double *volume, int nface, const int *face_cell,
                                  const double *face_geom, const double *cell_center, const double *face_center)
{
    if (!ctx) return GSIS_EINVAL;
    if (ctx->bound || ctx->meta_ready) return fail(ctx, GSIS_ESTATE, "set_spatial_mesh must precede workspace_size/bind");
    if (ctx->g.umesh) return fail(ctx, GSIS_ESTATE, "the spatial mesh is already set");
    if (!ctx->g.vlist) return fail(ctx, GSIS_ESTATE, "set_velocity_list must precede set_spatial_mesh");
    if (ctx->g.order != 1) return fail(ctx, GSIS_ESTATE, "an unstructured mesh runs the first-order update (order 1)");
    if (!ctx->mask.empty()) return fail(ctx, GSIS_ESTATE, "an unstructured mesh takes no solid mask");
    if (!volume || !face_cell || !face_geom) return fail(ctx, GSIS_EINVAL, "mesh array is NULL");
    if ((cell_center == nullptr) != (face_center == nullptr))
        return fail(ctx, GSIS_EINVAL, "give both cell and face centroids, or neither");
    if (ncell < 1 || nface < 1) return fail(ctx, GSIS_EINVAL, "the mesh needs cells and faces");
    if (ncell >= (1 << 23)) return fail(ctx, GSIS_EINVAL, "at most 2^23 - 1 cells");
    if ((long long)ncell * ctx->g.nv > (1ll << 40)) return fail(ctx, GSIS_EINVAL, "cells x nodes too large");
    for (int i = 0; i < ncell; ++i)
        if (!(volume[i] > 0) || !std::isfinite(volume[i])) return fail(ctx, GSIS_EINVAL, "cell volumes must be positive");
    std::vector<int> nfc(ncell, 0);
    std::vector<double> clos((size_t)ncell * 3, 0.0), area((size_t)ncell, 0.0);
    for (int f = 0; f < nface; ++f) {
        const int o = face_cell[2 * f], nb = face_cell[2 * f + 1];
        const double *gg = face_geom + (size_t)f * 4;
        if (o < 0 || o >= ncell || nb >= ncell || nb == o || nb < -NBC)
            return fail(ctx, GSIS_EINVAL, "face " + std::to_string(f) + ": bad owner or neighbour");
        if (!(gg[0] >= 0) || !std::isfinite(gg[0])) return fail(ctx, GSIS_EINVAL, "face areas must be >= 0");
        const double nn = gg[1] * gg[1] + gg[2] * gg[2] + gg[3] * gg[3];
        if (!(std::fabs(nn - 1.0) <= 1e-9)) return fail(ctx, GSIS_EINVAL, "face normals must be unit vectors");
        for (int side = 0; side < (nb >= 0 ? 2 : 1); ++side) {
            const int c = side ? nb : o;
            const double sg = side ? -1.0 : 1.0;
            if (++nfc[c] > UMAXF) return fail(ctx, GSIS_EINVAL, "a cell has more than 16 faces");
            for (int a = 0; a < 3; ++a) clos[(size_t)c * 3 + a] += sg * gg[0] * gg[1 + a];
            area[c] += gg[0];
        }
    }
    for (int i = 0; i < ncell; ++i) {
        const double *v = &clos[(size_t)i * 3];
        if (!(std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) <= 1e-9 * area[i]))
            return fail(ctx, GSIS_EINVAL, "cell " + std::to_string(i) + " is not closed (its area-weighted normals do not sum to zero)");
    }
    // face orientations up to sign, the three axes first (so that the classes
    // below refine the octants); a normal's canonical sign makes its first
    // component of magnitude above 1e-9 positive
    std::vector<double> ori = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
    std::vector<int> fk(nface), fflip(nface);
    for (int f = 0; f < nface; ++f) {
        const double *gg = face_geom + (size_t)f * 4 + 1;
        int a0 = 0;
        while (a0 < 2 && !(std::fabs(gg[a0]) > 1e-9)) ++a0;
        const double sg = gg[a0] < 0 ? -1.0 : 1.0;
        const double cn[3] = {sg * gg[0], sg * gg[1], sg * gg[2]};
        int k = 0;
        const int nk = (int)ori.size() / 4;
        for (; k < nk; ++k)
            if (std::fabs(ori[4 * k] - cn[0]) <= 1e-9 && std::fabs(ori[4 * k + 1] - cn[1]) <= 1e-9 &&
                std::fabs(ori[4 * k + 2] - cn[2]) <= 1e-9)
                break;
        if (k == nk) {
            if (nk == UMAXORI) return fail(ctx, GSIS_EINVAL, "the mesh has more than 32 distinct face orientations");
            ori.insert(ori.end(), {cn[0], cn[1], cn[2], 0.0});
        }
        fk[f] = k;
        fflip[f] = sg < 0 ? 1 : 0;
    }
    const int nori = (int)ori.size() / 4;
    // velocity classes: nodes with the same signs of xi . n_k for every k,
    // ordered by octant, then by mask; each class contiguous in a VDF row
    const int nv = ctx->g.nv;
    std::vector<unsigned> nmask(nv);
    for (int v = 0; v < nv; ++v) {
        const double *t = &ctx->vlist[(size_t)v * 4];
        unsigned m = 0;
        for (int k = 0; k < nori; ++k)
            if (t[0] * ori[4 * k] + t[1] * ori[4 * k + 1] + t[2] * ori[4 * k + 2] >= 0.0) m |= 1u << k;
        nmask[v] = m;
    }
    auto octant_of = [](unsigned m) { return (int)((~m) & 7u); };   // bit a of the mask: xi_a >= 0
    std::vector<unsigned> masks(nmask);
    std::sort(masks.begin(), masks.end(), [&](unsigned x, unsigned y) {
        return octant_of(x) != octant_of(y) ? octant_of(x) < octant_of(y) : x < y;
    });
    masks.erase(std::unique(masks.begin(), masks.end()), masks.end());
    const int ncls = (int)masks.size();
    if (ncls > 256) return fail(ctx, GSIS_EINVAL, "more than 256 velocity classes");
    std::map<unsigned, int> cls_of;
    for (int c = 0; c < ncls; ++c) cls_of[masks[c]] = c;
    std::vector<int> cnt(ncls, 0);
    for (int v = 0; v < nv; ++v) ++cnt[cls_of[nmask[v]]];
    if (*std::max_element(cnt.begin(), cnt.end()) > 65535 * 256)
        return fail(ctx, GSIS_EINVAL, "more than 65535 x 256 nodes in one velocity class");
    std::vector<int> cpos(ncls + 1, 0);
    for (int c = 0; c < ncls; ++c) cpos[c + 1] = cpos[c] + cnt[c];
    std::vector<int> perm(nv), at(cpos.begin(), cpos.end() - 1);
    for (int v = 0; v < nv; ++v) perm[at[cls_of[nmask[v]]]++] = v;
    // faces of every cell in input order (the owner's entry, then the neighbour's)
    std::vector<int> off(ncell + 1, 0);
    for (int i = 0; i < ncell; ++i) off[i + 1] = off[i] + nfc[i];
    if (off[ncell] >= (1 << 26)) return fail(ctx, GSIS_EINVAL, "at most 2^26 - 1 face entries (two per interior face)");
    std::vector<int> cnb(off[ncell]), cmeta(off[ncell]), pos(off.begin(), off.end() - 1);
    std::vector<double> cgeo((size_t)off[ncell] * 4);
    std::vector<int> bcell, bslot, bface, fcell((size_t)nface * 2), cface(off[ncell]);
    std::vector<double> bn;
    for (int f = 0; f < nface; ++f) {
        const int o = face_cell[2 * f], nb = face_cell[2 * f + 1];
        const double *gg = face_geom + (size_t)f * 4;
        int other = nb;
        int slot = 0;
        if (nb < 0) {
            slot = -1 - nb;
            other = -1 - (int)bcell.size();
            bcell.push_back(o);
            bslot.push_back(slot);
            bface.push_back(f);
            bn.insert(bn.end(), {gg[1], gg[2], gg[3], 0.0});
        }
        fcell[2 * (size_t)f] = o;
        fcell[2 * (size_t)f + 1] = other;
        cface[pos[o]] = f << 1;
        if (nb >= 0) cface[pos[nb]] = f << 1 | 1;
        int e = pos[o]++;
        cnb[e] = other;
        cmeta[e] = fk[f] | fflip[f] << 5 | slot << 6;
        cgeo[4 * (size_t)e] = gg[0] / volume[o];
        for (int a = 0; a < 3; ++a) cgeo[4 * (size_t)e + 1 + a] = gg[1 + a];
        if (nb >= 0) {
            e = pos[nb]++;
            cnb[e] = o;
            cmeta[e] = fk[f] | (fflip[f] ^ 1) << 5;
            cgeo[4 * (size_t)e] = gg[0] / volume[nb];
            for (int a = 0; a < 3; ++a) cgeo[4 * (size_t)e + 1 + a] = -gg[1 + a];
        }
    }
    // per class: the levels of its upwind graph (Kahn); then the sweep
    // entries level by level, classes in order, cells ascending
    std::vector<std::vector<int>> lev(ncls);
    int nlev = 0;
    std::vector<int> indeg(ncell), level(ncell);
    for (int c = 0; c < ncls; ++c) {
        const unsigned m = masks[c];
        auto leaves = [&](int i, int e) {   // the class's nodes leave cell i through entry e
            return (((m >> (cmeta[e] & 31)) & 1u) != 0) != (((cmeta[e] >> 5) & 1) != 0);
        };
        std::fill(indeg.begin(), indeg.end(), 0);
        for (int i = 0; i < ncell; ++i)
            for (int e = off[i]; e < off[i + 1]; ++e)
                if (cnb[e] >= 0 && !leaves(i, e)) ++indeg[i];
        std::vector<int> front, next;
        for (int i = 0; i < ncell; ++i)
            if (indeg[i] == 0) front.push_back(i);
        int done = 0, L = 0;
        while (!front.empty()) {
            std::sort(front.begin(), front.end());
            for (int i : front) level[i] = L;
            done += (int)front.size();
            next.clear();
            for (int i : front)
                for (int e = off[i]; e < off[i + 1]; ++e)
                    if (cnb[e] >= 0 && leaves(i, e) && --indeg[cnb[e]] == 0) next.push_back(cnb[e]);
            front.swap(next);
            ++L;
        }
        if (done < ncell)
            return fail(ctx, GSIS_EINVAL, "the upwind graph of velocity class " + std::to_string(c) +
                                              " has a cycle: no sweep order solves this mesh exactly");
        lev[c].assign(level.begin(), level.end());
        nlev = std::max(nlev, L);
    }
    std::vector<int> lcount(nlev + 1, 0);
    for (int c = 0; c < ncls; ++c)
        for (int i = 0; i < ncell; ++i) ++lcount[lev[c][i] + 1];
    for (int L = 0; L < nlev; ++L) lcount[L + 1] += lcount[L];
    std::vector<int> key(lcount[nlev]), lat(lcount.begin(), lcount.end() - 1);
    for (int c = 0; c < ncls; ++c)
        for (int i = 0; i < ncell; ++i) key[lat[lev[c][i]]++] = i << 8 | c;
    for (int L = 0; L < nlev; ++L)   // within a level: class by class, cells ascending
        std::sort(key.begin() + lcount[L], key.begin() + lcount[L + 1], [](int x, int y) {
            return (x & 255) != (y & 255) ? (x & 255) < (y & 255) : x < y;
        });
    std::vector<int> ent((size_t)lcount[nlev] * 2);
    for (size_t k = 0; k < key.size(); ++k) {
        const int i = key[k] >> 8;
        ent[2 * k] = key[k];
        ent[2 * k + 1] = off[i] << 5 | nfc[i];
    }
    // the macroscopic correction's geometry: least-squares weights of every
    // interior face entry, per face (S, n, h, |d|, d/|d|), the smallest h
    std::vector<double> lsq, fgeo;
    double hmin = 0.0;
    if (cell_center) {
        lsq.assign((size_t)off[ncell] * 3, 0.0);
        fgeo.assign((size_t)nface * 9, 0.0);
        hmin = INFINITY;
        for (int f = 0; f < nface; ++f) {
            const int o = face_cell[2 * f], nb = face_cell[2 * f + 1];
            const double *gg = face_geom + (size_t)f * 4, *xo = cell_center + (size_t)o * 3;
            const double *xr = nb >= 0 ? cell_center + (size_t)nb * 3 : face_center + (size_t)f * 3;
            const double k = nb >= 0 ? 1.0 : 2.0;
            double dv[3], dl = 0.0, h = 0.0;
            for (int a = 0; a < 3; ++a) {
                dv[a] = k * (xr[a] - xo[a]);
                dl += dv[a] * dv[a];
                h += dv[a] * gg[1 + a];
            }
            dl = std::sqrt(dl);
            if (!(h > 0.0) || !std::isfinite(h))
                return fail(ctx, GSIS_EINVAL, "face " + std::to_string(f) + ": its centroid distance along the normal is not positive");
            double *fg = &fgeo[(size_t)f * 9];
            fg[0] = gg[0];
            fg[1] = gg[1]; fg[2] = gg[2]; fg[3] = gg[3];
            fg[4] = h;
            fg[5] = dl;
            for (int a = 0; a < 3; ++a) fg[6 + a] = dv[a] / dl;
            hmin = std::min(hmin, h);
        }
        for (int i = 0; i < ncell; ++i) {
            double A[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, Ai[9];
            const double *xi = cell_center + (size_t)i * 3;
            for (int e = off[i]; e < off[i + 1]; ++e) {
                if (cnb[e] < 0) continue;
                const double *xj = cell_center + (size_t)cnb[e] * 3;
                for (int b = 0; b < 3; ++b)
                    for (int c = 0; c < 3; ++c) A[b * 3 + c] += (xj[b] - xi[b]) * (xj[c] - xi[c]);
            }
            sym3_pinv(A, Ai);
            for (int e = off[i]; e < off[i + 1]; ++e) {
                if (cnb[e] < 0) continue;
                const double *xj = cell_center + (size_t)cnb[e] * 3;
                for (int c = 0; c < 3; ++c) {
                    double acc = 0.0;
                    for (int k = 0; k < 3; ++k) acc += Ai[c * 3 + k] * (xj[k] - xi[k]);
                    lsq[(size_t)e * 3 + c] = acc;
                }
            }
        }
    }
    // commit
    Geo &g = ctx->g;
    ctx->uvol.assign(volume, volume + ncell);
    ctx->ucf_nb = cnb;
    ctx->ucf_meta = cmeta;
    ctx->ucf_g = cgeo;
    ctx->ucls.assign((size_t)ncls * 4, 0);
    for (int c = 0; c < ncls; ++c) {
        ctx->ucls[4 * c] = (int)masks[c];
        ctx->ucls[4 * c + 1] = cpos[c];
        ctx->ucls[4 * c + 2] = cnt[c];
    }
    ctx->ulev = ent;
    ctx->ulev_off = lcount;
    ctx->ubf_cell = bcell;
    ctx->ubf_slot = bslot;
    ctx->ubf_n = bn;
    ctx->uperm = perm;
    ctx->ucf_lsq = lsq;
    ctx->ucf_face = cface;
    ctx->ucf_first = off;
    ctx->ubf_face = bface;
    ctx->uf_cell = fcell;
    ctx->uf_geo = fgeo;
    g.ucen = cell_center ? 1 : 0;
    g.unface = nface;
    g.uhmin = hmin;
    g.umesh = 1;
    g.ucls = ncls;
    g.unbf = (int)bcell.size();
    g.nori = nori;
    g.umaxcnt = *std::max_element(cnt.begin(), cnt.end());
    g.umaxf = *std::max_element(nfc.begin(), nfc.end());
    g.nx = ncell;
    g.ny = g.nz = 1;
    g.ncell = ncell;
    ctx->mask.clear();
    return GSIS_OK;
}

gsis_status gsis_set_solid_mask(gsis_ctx *ctx, const uint8_t *mask, size_t n)
{
    if (!ctx) return GSIS_EINVAL;
    if (ctx->bound || ctx->meta_ready) return fail(ctx, GSIS_ESTATE, "set_solid_mask must precede workspace_size/bind");
    if (ctx->g.umesh) return fail(ctx, GSIS_ESTATE, "an unstructured mesh takes no solid mask (leave solid cells out of it)");
    if (!mask) return fail(ctx, GSIS_EINVAL, "mask is NULL");
    if (n != (size_t)ctx->g.ncell) return fail(ctx, GSIS_EINVAL, "mask size must be nx*ny*nz");
    size_t fluid = 0;
    for (size_t i = 0; i < n; ++i) {
        if (mask[i] > 1) return fail(ctx, GSIS_EINVAL, "mask entries must be 0 or 1");
        fluid += mask[i] == 0;
    }
    if (fluid == 0) return fail(ctx, GSIS_EINVAL, "all cells are solid");
    ctx->mask.assign(mask, mask + n);
    return GSIS_OK;
}

gsis_status gsis_set_boundary(gsis_ctx *ctx, int face, int kind, const double u[3], double T, double rho)
{
    if (!ctx) return GSIS_EINVAL;
    if (ctx->bound) return fail(ctx, GSIS_ESTATE, "set_boundary must precede bind_workspace");
    if (face < 0 || face >= NBC) return fail(ctx, GSIS_EINVAL, "face must be 0..6");
    if (kind != GSIS_DIFFUSE_WALL && kind != GSIS_MAXWELL_INFLOW) return fail(ctx, GSIS_EINVAL, "unknown boundary kind");
    if (!finite3(u)) return fail(ctx, GSIS_EINVAL, "boundary velocity must be finite");
    if (!(T > 0) || !std::isfinite(T)) return fail(ctx, GSIS_EINVAL, "boundary temperature must be positive");
    if (kind == GSIS_MAXWELL_INFLOW && (!(rho >= 0) || !std::isfinite(rho)))
        return fail(ctx, GSIS_EINVAL, "inflow density must be >= 0");
    ctx->bc.kind[face] = kind;
    for (int a = 0; a < 3; ++a) ctx->bc.u[face][a] = u[a];
    ctx->bc.T[face] = T;
    ctx->bc.rho[face] = kind == GSIS_MAXWELL_INFLOW ? rho : 1.0;
    return GSIS_OK;
}

gsis_status gsis_set_wall_flux(gsis_ctx *ctx, int model)
{
    if (!ctx) return GSIS_EINVAL;
    if (ctx->bound) return fail(ctx, GSIS_ESTATE, "set_wall_flux must precede bind_workspace");
    if (model != GSIS_WALLFLUX_MAXWELL && model != GSIS_WALLFLUX_G13) return fail(ctx, GSIS_EINVAL, "unknown wall flux model");
    ctx->g.wall_flux = model;
    return GSIS_OK;
}

gsis_status gsis_workspace_size(const gsis_ctx *cctx, size_t *bytes)
{
    gsis_ctx *ctx = const_cast<gsis_ctx *>(cctx);
    if (!ctx || !bytes) return GSIS_EINVAL;
    if (!ctx->meta_ready) build_meta(ctx);
    Dev save = ctx->d;
    *bytes = layout(ctx, nullptr);
    ctx->d = save;
    return GSIS_OK;
}

gsis_status gsis_bind_workspace(gsis_ctx *ctx, void *device_ptr, size_t bytes)
{
    if (!ctx) return GSIS_EINVAL;
    if (ctx->bound) return fail(ctx, GSIS_ESTATE, "workspace already bound");
    if (!device_ptr) return fail(ctx, GSIS_EINVAL, "workspace pointer is NULL");
    if ((uintptr_t)device_ptr % 256) return fail(ctx, GSIS_EINVAL, "workspace must be 256-byte aligned");
    if (!ctx->meta_ready) build_meta(ctx);
    size_t need = layout(ctx, nullptr);
    if (bytes < need) return fail(ctx, GSIS_ENOMEM, "workspace smaller than gsis_workspace_size");
    ctx->ws = (char *)device_ptr;
    ctx->ws_bytes = bytes;
    layout(ctx, ctx->ws);
    const Geo &g = ctx->g;
    Dev &d = ctx->d;
    auto up = [&](void *dst, const void *src, size_t nbytes) { return hipMemcpy(dst, src, nbytes, hipMemcpyHostToDevice); };
    HIPCHK(ctx, up(d.cflag, ctx->cflag.data(), ctx->cflag.size() * sizeof(int)));
    {
        // the device copy is direction-major, [6][ncell], so a wave of consecutive cells reads consecutive words
        std::vector<int> nt(ctx->nbr.size());
        for (int cell = 0; cell < g.ncell; ++cell)
            for (int dir = 0; dir < 6; ++dir) nt[(size_t)dir * g.ncell + cell] = ctx->nbr[(size_t)cell * 6 + dir];
        HIPCHK(ctx, up(d.nbr, nt.data(), nt.size() * sizeof(int)));
    }
    if (g.nface > 0) {
        HIPCHK(ctx, up(d.face_cell, ctx->face_cell.data(), g.nface * sizeof(int)));
        HIPCHK(ctx, up(d.face_dir, ctx->face_dir.data(), g.nface * sizeof(int)));
        HIPCHK(ctx, up(d.face_bc, ctx->face_bc.data(), g.nface * sizeof(int)));
    }
    if (!g.vlist) {
        // per-axis tables of the separable kernels (tensor grid)
        std::vector<double> xt((size_t)g.n1[0] * 4), yt((size_t)g.n1[1] * 2), zt((size_t)g.n1[2] * 2);
        for (int a = 0; a < 3; ++a) {
            std::vector<float> x32(ctx->xi[a].begin(), ctx->xi[a].end());
            HIPCHK(ctx, up(d.xi64[a], ctx->xi[a].data(), g.n1[a] * sizeof(double)));
            HIPCHK(ctx, up(d.xi32[a], x32.data(), g.n1[a] * sizeof(float)));
            HIPCHK(ctx, up(d.w64[a], ctx->w[a].data(), g.n1[a] * sizeof(double)));
        }
        for (int k = 0; k < g.n1[0]; ++k) {
            double x = ctx->xi[0][k], w = ctx->w[0][k];
            xt[4 * k] = w; xt[4 * k + 1] = w * x; xt[4 * k + 2] = w * x * x; xt[4 * k + 3] = w * x * x * x;
        }
        for (int k = 0; k < g.n1[1]; ++k) { yt[2 * k] = ctx->w[1][k]; yt[2 * k + 1] = ctx->xi[1][k]; }
        for (int k = 0; k < g.n1[2]; ++k) { zt[2 * k] = ctx->w[2][k]; zt[2 * k + 1] = ctx->xi[2][k]; }
        HIPCHK(ctx, up(d.xtab, xt.data(), xt.size() * sizeof(double)));
        HIPCHK(ctx, up(d.ytab, yt.data(), yt.size() * sizeof(double)));
        HIPCHK(ctx, up(d.ztab, zt.data(), zt.size() * sizeof(double)));
    }
    {
        // every node in the internal order: (xi_x, xi_y, xi_z, weight)
        std::vector<double> nt((size_t)g.nv * 4);
        std::vector<float> nt32((size_t)g.nv * 4);
        for (int i = 0; i < g.nv; ++i) {
            const int k = ctx->perm[i];
            double *t = &nt[(size_t)i * 4];
            if (g.vlist) {
                for (int q = 0; q < 4; ++q) t[q] = ctx->vlist[(size_t)k * 4 + q];
            } else {
                const int kx = k % g.n1[0], ky = (k / g.n1[0]) % g.n1[1], kz = k / (g.n1[0] * g.n1[1]);
                t[0] = ctx->xi[0][kx];
                t[1] = ctx->xi[1][ky];
                t[2] = ctx->xi[2][kz];
                t[3] = ctx->w[0][kx] * ctx->w[1][ky] * ctx->w[2][kz];
            }
            for (int q = 0; q < 4; ++q) nt32[(size_t)i * 4 + q] = (float)t[q];
        }
        HIPCHK(ctx, up(d.nt64, nt.data(), nt.size() * sizeof(double)));
        HIPCHK(ctx, up(d.nt32, nt32.data(), nt32.size() * sizeof(float)));
    }
    HIPCHK(ctx, up(d.perm, ctx->perm.data(), ctx->perm.size() * sizeof(int)));
    if (g.umesh) {
        std::vector<float> g32(ctx->ucf_g.begin(), ctx->ucf_g.end());
        HIPCHK(ctx, up(d.uvol, ctx->uvol.data(), ctx->uvol.size() * sizeof(double)));
        HIPCHK(ctx, up(d.ucf_nb, ctx->ucf_nb.data(), ctx->ucf_nb.size() * sizeof(int)));
        HIPCHK(ctx, up(d.ucf_meta, ctx->ucf_meta.data(), ctx->ucf_meta.size() * sizeof(int)));
        HIPCHK(ctx, up(d.ucf_g64, ctx->ucf_g.data(), ctx->ucf_g.size() * sizeof(double)));
        HIPCHK(ctx, up(d.ucf_g32, g32.data(), g32.size() * sizeof(float)));
        HIPCHK(ctx, up(d.ucls, ctx->ucls.data(), ctx->ucls.size() * sizeof(int)));
        HIPCHK(ctx, up(d.ulev, ctx->ulev.data(), ctx->ulev.size() * sizeof(int)));
        if (g.ucen) {
            HIPCHK(ctx, up(d.ucf_lsq, ctx->ucf_lsq.data(), ctx->ucf_lsq.size() * sizeof(double)));
            HIPCHK(ctx, up(d.ucf_face, ctx->ucf_face.data(), ctx->ucf_face.size() * sizeof(int)));
            HIPCHK(ctx, up(d.ucf_first, ctx->ucf_first.data(), ctx->ucf_first.size() * sizeof(int)));
            if (g.unbf > 0) HIPCHK(ctx, up(d.ubf_face, ctx->ubf_face.data(), ctx->ubf_face.size() * sizeof(int)));
            HIPCHK(ctx, up(d.uf_cell, ctx->uf_cell.data(), ctx->uf_cell.size() * sizeof(int)));
            HIPCHK(ctx, up(d.uf_geo, ctx->uf_geo.data(), ctx->uf_geo.size() * sizeof(double)));
        }
        if (g.unbf > 0) {
            HIPCHK(ctx, up(d.ubf_cell, ctx->ubf_cell.data(), ctx->ubf_cell.size() * sizeof(int)));
            HIPCHK(ctx, up(d.ubf_slot, ctx->ubf_slot.data(), ctx->ubf_slot.size() * sizeof(int)));
            HIPCHK(ctx, up(d.ubf_n, ctx->ubf_n.data(), ctx->ubf_n.size() * sizeof(double)));
        }
    }
    HIPCHK(ctx, upload_tiles(ctx));
    HIPCHK(ctx, hipMemset(d.errflag, 0, 4 * sizeof(int)));
    HIPCHK(ctx, hipMemset(d.dmax, 0, (size_t)2 * DSLOT * DSTRIDE * sizeof(unsigned long long)));
    HIPCHK(ctx, launch_setup_tables(g, ctx->bc, d, nullptr));
    HIPCHK(ctx, hipDeviceSynchronize());
    ctx->bound = true;
    return GSIS_OK;
}

gsis_status gsis_set_stream(gsis_ctx *ctx, void *hip_stream)
{
    if (!ctx) return GSIS_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
    return GSIS_OK;
}

gsis_status gsis_init_maxwellian(gsis_ctx *ctx, double rho, const double u[3], double T, double Tr)
{
    if (!ctx) return GSIS_EINVAL;
    if (!ctx->bound) return fail(ctx, GSIS_ESTATE, "bind_workspace first");
    if (!(rho > 0) || !std::isfinite(rho) || !(T > 0) || !std::isfinite(T) || !finite3(u))
        return fail(ctx, GSIS_EINVAL, "init needs rho > 0, T > 0, finite u");
    if (ctx->g.species == GSIS_DIATOMIC && (!(Tr > 0) || !std::isfinite(Tr)))
        return fail(ctx, GSIS_EINVAL, "init needs Tr > 0");
    gsis_status st = reset_flags(ctx);
    if (st) return st;
    HIPCHK(ctx, launch_init_maxwellian(ctx->g, ctx->d, ctx->fp32, rho, u, T, Tr, ctx->stream));
    if ((st = reduce_vdf(ctx))) return st;
    HIPCHK(ctx, launch_snapshot(target_of(ctx), ctx->stream));
    ctx->pending = false;
    ctx->inited = true;
    ctx->stepped = false;
    ctx->passes = 0;
    ctx->watch = DivWatch();
    return GSIS_OK;
}

gsis_status gsis_kinetic_step(gsis_ctx *ctx, int npasses)
{
    if (!ctx) return GSIS_EINVAL;
    if (!ctx->inited) return fail(ctx, GSIS_ESTATE, "initialise the VDF first");
    if (npasses < 0) return fail(ctx, GSIS_EINVAL, "npasses must be >= 0");
    const Geo &g = ctx->g;
    const Target t = target_of(ctx);
    for (int n = 0; n < npasses; ++n) {
        if (g.inv_dt != 0.0 || g.order == 2) {   // the pass reads f^n pointwise
            gsis_status st = materialize(ctx);
            if (st) return st;
        }
        PhaseTimer t0, t1, t2, t3;
        if (g.umesh) {
            HIPCHK(ctx, t0.start(ctx, GSIS_PHASE_PREP));
            HIPCHK(ctx, launch_params(t, ctx->stream));
            HIPCHK(ctx, launch_uface_scale(t, ctx->pending ? 1 : 0, ctx->stream));
            HIPCHK(ctx, t0.stop());
            HIPCHK(ctx, t1.start(ctx, GSIS_PHASE_SWEEP));
            HIPCHK(ctx, launch_usweep(t, ctx->ulev_off.data(), (int)ctx->ulev_off.size() - 1, ctx->stream));
            HIPCHK(ctx, t1.stop());
            ctx->pending = false;   // every point was rewritten
            HIPCHK(ctx, t2.start(ctx, GSIS_PHASE_MOMENTS));
            gsis_status st = reduce_vdf(ctx);
            if (st) return st;
            HIPCHK(ctx, t2.stop());
            ctx->passes++;
            ctx->stepped = true;
            continue;
        }
        HIPCHK(ctx, t0.start(ctx, GSIS_PHASE_PREP));
        HIPCHK(ctx, launch_params(t, ctx->stream));
        HIPCHK(ctx, launch_face_scale(t, ctx->stream));
        HIPCHK(ctx, t0.stop());
        if (g.order == 2) {
            HIPCHK(ctx, t3.start(ctx, GSIS_PHASE_RECON));
            HIPCHK(ctx, launch_recon(g, ctx->d, ctx->fp32, ctx->stream));
            HIPCHK(ctx, t3.stop());
        }
        HIPCHK(ctx, t1.start(ctx, GSIS_PHASE_SWEEP));
        HIPCHK(ctx, launch_sweep(t, ctx->stream));
        HIPCHK(ctx, t1.stop());
        ctx->pending = false;   // every fluid point was rewritten
        HIPCHK(ctx, t2.start(ctx, GSIS_PHASE_MOMENTS));
        gsis_status st = reduce_vdf(ctx);
        if (st) return st;
        HIPCHK(ctx, t2.stop());
        ctx->passes++;
        ctx->stepped = true;
    }
    return GSIS_OK;
}

gsis_status gsis_moments(gsis_ctx *ctx, double *out, int out_is_device)
{
    if (!ctx) return GSIS_EINVAL;
    if (!ctx->inited) return fail(ctx, GSIS_ESTATE, "initialise the VDF first");
    if (!out) return fail(ctx, GSIS_EINVAL, "out is NULL");
    size_t nm = ctx->g.species == GSIS_DIATOMIC ? GSIS_NMOM_DIATOMIC : GSIS_NMOM_MONATOMIC;
    HIPCHK(ctx, hipMemcpy2DAsync(out, nm * sizeof(double), ctx->d.cm, NMOM * sizeof(double), nm * sizeof(double),
                                 ctx->g.ncell, out_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                 ctx->stream));
    if (!out_is_device) HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return GSIS_OK;
}

gsis_status gsis_gsis_correct(gsis_ctx *ctx, int inner_iters)
{
    if (!ctx) return GSIS_EINVAL;
    if (ctx->g.umesh && !ctx->g.ucen)
        return fail(ctx, GSIS_ESTATE, "the macroscopic correction on an unstructured mesh needs its centroids");
    if (!ctx->inited || !ctx->stepped) return fail(ctx, GSIS_ESTATE, "gsis_correct needs a kinetic step since init");
    if (inner_iters < 0) return fail(ctx, GSIS_EINVAL, "inner_iters must be >= 0");
    gsis_status st = materialize(ctx);
    if (st) return st;
    PhaseTimer t;
    HIPCHK(ctx, t.start(ctx, GSIS_PHASE_MACRO));
    const Target tg = target_of(ctx);
    if (ctx->g.umesh) HIPCHK(ctx, launch_umacro(tg, inner_iters, ctx->stream));
    else HIPCHK(ctx, launch_gsis_macro(tg, inner_iters, ctx->stream));
    HIPCHK(ctx, launch_commit_correction(tg, ctx->stream));
    HIPCHK(ctx, launch_derive(tg, ctx->stream));
    HIPCHK(ctx, t.stop());
    ctx->pending = true;
    return GSIS_OK;
}

gsis_status gsis_precondition(gsis_ctx *ctx, int macro_steps, int kinetic_steps)
{
    if (!ctx) return GSIS_EINVAL;
    if (ctx->g.umesh && !ctx->g.ucen)
        return fail(ctx, GSIS_ESTATE, "the Euler steps on an unstructured mesh need its centroids");
    if (!ctx->inited) return fail(ctx, GSIS_ESTATE, "initialise the VDF first");
    if (macro_steps < 0 || kinetic_steps < 0) return fail(ctx, GSIS_EINVAL, "steps must be >= 0");
    gsis_status st = materialize(ctx);
    if (st) return st;
    {
        PhaseTimer t;
        HIPCHK(ctx, t.start(ctx, GSIS_PHASE_MACRO));
        const Target tg = target_of(ctx);
        if (ctx->g.umesh) HIPCHK(ctx, launch_umacro(tg, macro_steps, ctx->stream, 1));
        else HIPCHK(ctx, launch_gsis_macro(tg, macro_steps, ctx->stream, 1));
        HIPCHK(ctx, launch_commit_correction(tg, ctx->stream));
        HIPCHK(ctx, launch_derive(tg, ctx->stream));
        HIPCHK(ctx, t.stop());
    }
    ctx->pending = true;
    return gsis_kinetic_step(ctx, kinetic_steps);
}

gsis_status gsis_residual(gsis_ctx *ctx, double eps[3])
{
    if (!ctx) return GSIS_EINVAL;
    if (!ctx->inited) return fail(ctx, GSIS_ESTATE, "initialise the VDF first");
    if (!eps) return fail(ctx, GSIS_EINVAL, "eps is NULL");
    PhaseTimer t;
    HIPCHK(ctx, t.start(ctx, GSIS_PHASE_RESIDUAL));
    HIPCHK(ctx, launch_residual(target_of(ctx), ctx->stream));
    double *total = ctx->d.red + (size_t)resid_blocks(ctx->g) * 6;
    return residual_finish(ctx, total, &t, eps);
}

gsis_status gsis_residual_noalloc(gsis_ctx *ctx, double eps[3])
{
    if (!ctx) return GSIS_EINVAL;
    if (resid_blocks(ctx->g) > RESID_STATIC_BLOCKS)
        return fail(ctx, GSIS_EINVAL, "gsis_residual_noalloc takes at most " +
                                          std::to_string((long long)RESID_STATIC_BLOCKS * 256) + " cells");
    if (!ctx->inited) return fail(ctx, GSIS_ESTATE, "initialise the VDF first");
    if (!eps) return fail(ctx, GSIS_EINVAL, "eps is NULL");
    double *red = nullptr;
    HIPCHK(ctx, resid_static_scratch(&red));
    HIPCHK(ctx, launch_residual(target_of(ctx), ctx->stream, red));
    return residual_finish(ctx, red + (size_t)resid_blocks(ctx->g) * 6, nullptr, eps);
}

gsis_status gsis_get_vdf(gsis_ctx *ctx, double *f0_device, double *f1_device)
{
    if (!ctx) return GSIS_EINVAL;
    if (!ctx->inited) return fail(ctx, GSIS_ESTATE, "initialise the VDF first");
    if (!f0_device || (ctx->g.species == GSIS_DIATOMIC && !f1_device)) return fail(ctx, GSIS_EINVAL, "NULL output");
    gsis_status st = materialize(ctx);
    if (st) return st;
    HIPCHK(ctx, launch_to_canonical(ctx->g, ctx->d, ctx->fp32, ctx->d.f0, f0_device, ctx->stream));
    if (ctx->g.species == GSIS_DIATOMIC)
        HIPCHK(ctx, launch_to_canonical(ctx->g, ctx->d, ctx->fp32, ctx->d.f1, f1_device, ctx->stream));
    return GSIS_OK;
}

gsis_status gsis_set_vdf(gsis_ctx *ctx, const double *f0_device, const double *f1_device)
{
    if (!ctx) return GSIS_EINVAL;
    if (!ctx->bound) return fail(ctx, GSIS_ESTATE, "bind_workspace first");
    if (!f0_device || (ctx->g.species == GSIS_DIATOMIC && !f1_device)) return fail(ctx, GSIS_EINVAL, "NULL input");
    gsis_status st = reset_flags(ctx);
    if (st) return st;
    HIPCHK(ctx, launch_from_canonical(ctx->g, ctx->d, ctx->fp32, f0_device, ctx->d.f0, ctx->stream));
    if (ctx->g.species == GSIS_DIATOMIC)
        HIPCHK(ctx, launch_from_canonical(ctx->g, ctx->d, ctx->fp32, f1_device, ctx->d.f1, ctx->stream));
    if ((st = reduce_vdf(ctx))) return st;
    HIPCHK(ctx, launch_snapshot(target_of(ctx), ctx->stream));
    ctx->pending = false;
    ctx->inited = true;
    ctx->stepped = false;
    ctx->passes = 0;
    ctx->watch = DivWatch();
    return GSIS_OK;
}

gsis_status gsis_state_size(const gsis_ctx *ctx, size_t *bytes)
{
    if (!ctx || !bytes) return GSIS_EINVAL;
    if (!ctx->bound) return fail(const_cast<gsis_ctx *>(ctx), GSIS_ESTATE, "bind_workspace first");
    std::vector<StatePart> parts;
    state_parts(ctx, parts);
    size_t off = align256(sizeof(StateHeader));
    for (auto &p : parts) off = align256(off + p.bytes);
    *bytes = off;
    return GSIS_OK;
}

gsis_status gsis_get_state(gsis_ctx *ctx, void *dst_device)
{
    if (!ctx) return GSIS_EINVAL;
    if (!ctx->inited) return fail(ctx, GSIS_ESTATE, "initialise the VDF first");
    if (!dst_device) return fail(ctx, GSIS_EINVAL, "NULL destination");
    StateHeader h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, "GSISSTA", 8);
    h.version = 2;
    h.ncell = ctx->g.ncell;
    h.nv = ctx->g.nv;
    h.fp32 = ctx->fp32;
    h.species = ctx->g.species;
    h.pending = ctx->pending;
    h.stepped = ctx->stepped;
    h.have_first = 0;
    h.passes = ctx->passes;
    for (int k = 0; k < 3; ++k) {
        h.have_first |= ctx->watch.have[k] ? 1 << k : 0;
        h.first_eps[k] = ctx->watch.first[k];
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(dst_device, &h, sizeof h, hipMemcpyHostToDevice));
    std::vector<StatePart> parts;
    state_parts(ctx, parts);
    size_t off = align256(sizeof(StateHeader));
    for (auto &p : parts) {
        HIPCHK(ctx, hipMemcpyAsync((char *)dst_device + off, p.ptr, p.bytes, hipMemcpyDeviceToDevice, ctx->stream));
        off = align256(off + p.bytes);
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return GSIS_OK;
}

gsis_status gsis_set_state(gsis_ctx *ctx, const void *src_device)
{
    if (!ctx) return GSIS_EINVAL;
    if (!ctx->bound) return fail(ctx, GSIS_ESTATE, "bind_workspace first");
    if (!src_device) return fail(ctx, GSIS_EINVAL, "NULL source");
    StateHeader h;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(&h, src_device, sizeof h, hipMemcpyDeviceToHost));
    if (std::memcmp(h.magic, "GSISSTA", 8) != 0 || h.version != 2 || h.ncell != ctx->g.ncell || h.nv != ctx->g.nv ||
        h.fp32 != (int)ctx->fp32 || h.species != ctx->g.species)
        return fail(ctx, GSIS_EINVAL, "state blob does not match this context");
    std::vector<StatePart> parts;
    state_parts(ctx, parts);
    size_t off = align256(sizeof(StateHeader));
    for (auto &p : parts) {
        HIPCHK(ctx, hipMemcpyAsync(p.ptr, (const char *)src_device + off, p.bytes, hipMemcpyDeviceToDevice, ctx->stream));
        off = align256(off + p.bytes);
    }
    gsis_status st = reset_flags(ctx);
    if (st) return st;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->pending = h.pending != 0;
    ctx->stepped = h.stepped != 0;
    ctx->passes = h.passes;
    for (int k = 0; k < 3; ++k) {
        ctx->watch.have[k] = (h.have_first >> k) & 1;
        ctx->watch.first[k] = h.first_eps[k];
    }
    ctx->inited = true;
    return GSIS_OK;
}

gsis_status gsis_set_tile(gsis_ctx *ctx, int tx, int ty, int tz, int block)
{
    if (!ctx) return GSIS_EINVAL;
    if (ctx->g.umesh) return fail(ctx, GSIS_ESTATE, "an unstructured mesh has no sweep tiles");
    if (tx == 0 && ty == 0 && tz == 0 && block == 0) {
        default_tile(ctx);
    } else {
        if (!sweep_shape_supported(ctx->fp32, ctx->g.species == GSIS_DIATOMIC, tx, ty))
            return fail(ctx, GSIS_EINVAL, "tile (tx, ty) not compiled for this precision and gas");
        if (tz < 1 || tz > 1024) return fail(ctx, GSIS_EINVAL, "tz must be 1..1024");
        const int nw = sweep_shape_waves(ctx->fp32, tx, ty);
        if (nw > 1 && block != 64 * nw) return fail(ctx, GSIS_EINVAL, "block must be 64 x the waves of this tile's wave grid");
        if (nw == 1 && block != 64 && block != 128 && block != 256) return fail(ctx, GSIS_EINVAL, "block must be 64, 128 or 256");
        int ntx = (ctx->g.nx + tx - 1) / tx, nty = (ctx->g.ny + ty - 1) / ty, ntz = (ctx->g.nz + tz - 1) / tz;
        if (ntx > 1023 || nty > 1023 || ntz > 1023) return fail(ctx, GSIS_EINVAL, "too many tiles per axis");
        ctx->tx = tx; ctx->ty = ty; ctx->tz = tz; ctx->bs = block;
    }
    if (ctx->meta_ready) build_tiles(ctx);
    if (ctx->bound) HIPCHK(ctx, upload_tiles(ctx));
    return GSIS_OK;
}

gsis_status gsis_autotune(gsis_ctx *ctx, int reps, int *cfg_out, double *ms_out, int max, int *count)
{
    if (!ctx) return GSIS_EINVAL;
    if (ctx->g.umesh) return fail(ctx, GSIS_ESTATE, "an unstructured mesh has no sweep tiles to tune");
    if (!ctx->inited) return fail(ctx, GSIS_ESTATE, "initialise the VDF first");
    if (reps < 1 || max < 0) return fail(ctx, GSIS_EINVAL, "reps must be >= 1");
    if (ctx->g.inv_dt != 0.0 || ctx->g.order != 1)
        return fail(ctx, GSIS_EINVAL, "autotune needs the first-order source iteration (inv_dt = 0, order 1)");
    const Geo &g = ctx->g;
    bool dia = g.species == GSIS_DIATOMIC;
    int shapes[32];
    int nsh = sweep_shapes(ctx->fp32, shapes, 16);
    struct Cand { int tx, ty, tz, bs; double ms; };
    std::vector<Cand> cands;
    for (int k = 0; k < nsh; ++k) {
        int tx = shapes[2 * k], ty = shapes[2 * k + 1];
        if (!sweep_shape_supported(ctx->fp32, dia, tx, ty)) continue;
        const int nw = sweep_shape_waves(ctx->fp32, tx, ty);
        for (int tz : {tx / 2, tx, 2 * tx, 4 * tx})
            for (int bs : {64, 128, 256})
                if (nw == 1 || bs == 64 * nw) cands.push_back({tx, ty, std::max(tz, 1), bs, 0.0});
    }
    int save[4] = {ctx->tx, ctx->ty, ctx->tz, ctx->bs};
    {
        const Target t0 = target_of(ctx);
        HIPCHK(ctx, launch_params(t0, ctx->stream));
        HIPCHK(ctx, launch_face_scale(t0, ctx->stream));
    }
    hipEvent_t e0, e1;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    gsis_status st = GSIS_OK;
    for (auto &c : cands) {
        ctx->tx = c.tx; ctx->ty = c.ty; ctx->tz = c.tz; ctx->bs = c.bs;
        build_tiles(ctx);
        hipError_t e = upload_tiles(ctx);
        const Target tc = target_of(ctx);
        if (e == hipSuccess) e = launch_sweep(tc, ctx->stream);   // warm-up launch of this configuration
        if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_sweep(tc, ctx->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) { st = fail(ctx, GSIS_EDEVICE, std::string("autotune: ") + hipGetErrorString(e)); break; }
        c.ms = ms / reps;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st) {
        ctx->tx = save[0]; ctx->ty = save[1]; ctx->tz = save[2]; ctx->bs = save[3];
        build_tiles(ctx);
        upload_tiles(ctx);
        return st;
    }
    size_t best = 0;
    for (size_t k = 1; k < cands.size(); ++k)
        if (cands[k].ms < cands[best].ms) best = k;
    ctx->tx = cands[best].tx; ctx->ty = cands[best].ty; ctx->tz = cands[best].tz; ctx->bs = cands[best].bs;
    build_tiles(ctx);
    HIPCHK(ctx, upload_tiles(ctx));
    // the VDF now holds this pass's sweep result (identical under every configuration)
    ctx->pending = false;
    st = reduce_vdf(ctx);
    if (st) return st;
    ctx->passes++;
    ctx->stepped = true;
    int n = 0;
    for (size_t k = 0; k < cands.size() && n < max; ++k, ++n) {
        if (cfg_out) {
            cfg_out[4 * n] = cands[k].tx; cfg_out[4 * n + 1] = cands[k].ty;
            cfg_out[4 * n + 2] = cands[k].tz; cfg_out[4 * n + 3] = cands[k].bs;
        }
        if (ms_out) ms_out[n] = cands[k].ms;
    }
    if (count) *count = n;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return GSIS_OK;
}

gsis_status gsis_get_tile(const gsis_ctx *ctx, int *tile)
{
    if (!ctx || !tile) return GSIS_EINVAL;
    tile[0] = ctx->tx; tile[1] = ctx->ty; tile[2] = ctx->tz; tile[3] = ctx->bs;
    return GSIS_OK;
}

gsis_status gsis_tile_shapes(int *out, int max, int *count)
{
    if (!out || !count || max < 0) return GSIS_EINVAL;
    int buf[64];
    int n32 = sweep_shapes(true, buf, 16);
    int n64 = sweep_shapes(false, buf + 2 * n32, 16);
    int n = 0;
    for (int k = 0; k < n32 + n64 && n < max; ++k) {
        out[3 * n] = buf[2 * k];
        out[3 * n + 1] = buf[2 * k + 1];
        out[3 * n + 2] = k < n32 ? 32 : 64;
        ++n;
    }
    *count = n;
    return GSIS_OK;
}

gsis_status gsis_get_vdf_nodes(gsis_ctx *ctx, const int *nodes, int nnodes, double *out_device)
{
    if (!ctx) return GSIS_EINVAL;
    if (!ctx->inited) return fail(ctx, GSIS_ESTATE, "initialise the VDF first");
    if (!nodes || nnodes < 1 || nnodes > 4096 || !out_device) return fail(ctx, GSIS_EINVAL, "bad node list");
    std::vector<int> inv(ctx->g.nv);
    for (int k = 0; k < ctx->g.nv; ++k) inv[ctx->perm[k]] = k;
    std::vector<int> internal(nnodes);
    for (int k = 0; k < nnodes; ++k) {
        if (nodes[k] < 0 || nodes[k] >= ctx->g.nv) return fail(ctx, GSIS_EINVAL, "node index out of range");
        internal[k] = inv[nodes[k]];
    }
    gsis_status st = materialize(ctx);
    if (st) return st;
    for (int k = 0; k < nnodes; ++k)
        HIPCHK(ctx, launch_vdf_node(ctx->g, ctx->d, ctx->fp32, internal[k], out_device + (size_t)k * ctx->g.ncell,
                                    ctx->stream));
    return GSIS_OK;
}

gsis_status gsis_profile_enable(gsis_ctx *ctx, int enable)
{
    if (!ctx) return GSIS_EINVAL;
    ctx->prof = enable != 0;
    return GSIS_OK;
}

gsis_status gsis_profile_read(gsis_ctx *ctx, double *ms, long long *calls, int reset)
{
    if (!ctx || !ms || !calls) return GSIS_EINVAL;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (auto &e : ctx->ev_open) {
        float t = 0.0f;
        HIPCHK(ctx, hipEventElapsedTime(&t, e.second.first, e.second.second));
        ctx->prof_ms[e.first] += t;
        ctx->prof_calls[e.first] += 1;
        ctx->ev_pool.push_back(e.second.first);
        ctx->ev_pool.push_back(e.second.second);
    }
    ctx->ev_open.clear();
    for (int k = 0; k < GSIS_NPHASE; ++k) {
        ms[k] = ctx->prof_ms[k];
        calls[k] = ctx->prof_calls[k];
        if (reset) { ctx->prof_ms[k] = 0.0; ctx->prof_calls[k] = 0; }
    }
    return GSIS_OK;
}

gsis_status gsis_pass_count(const gsis_ctx *ctx, long long *passes)
{
    if (!ctx || !passes) return GSIS_EINVAL;
    *passes = ctx->passes;
    return GSIS_OK;
}

}  // extern "C"

// ====================================================================== batches

struct gsis_batch {
    std::vector<gsis_ctx *> cs;
    hipStream_t stream = nullptr;
    bool bound = false, inited = false;
    bool fp32 = false, dia = false;
    int tx = 4, ty = 4, tz = 4, bs = 128;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Case *dcases = nullptr;        // device case table
    int2 *dmap = nullptr;          // device block maps
    size_t map_cap = 0;
    double *hist = nullptr;        // [hist_cap][ncase][6] residual sums
    int *hist_ctr = nullptr;
    int hist_cap = 1024;
    std::vector<size_t> case_off;  // workspace offset of every case
    std::vector<Case> hcases;
    std::vector<int2> hmap;
    std::vector<const int2 *> pmap;
    std::vector<int> npblk;
    Target t;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_inner = -1;
    long long iters_run = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed = false;
    std::string err;
    void drop_graph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        graph_inner = -1;
    }
    ~gsis_batch()
    {
        drop_graph();
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
    }
};

namespace {

gsis_status bfail(gsis_batch *b, gsis_status s, const std::string &msg)
{
    if (b) b->err = msg;
    return s;
}

#define BHIPCHK(b, expr)                                                                               \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return bfail(b, GSIS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Upper bound of the block-map entries: every launch kind, plus the sweep at
// its finest tiling (4 x 4 x 1 tiles, 64-thread blocks).
size_t batch_map_cap(const gsis_batch *b)
{
    size_t n = 0;
    for (const gsis_ctx *c : b->cs) {
        for (int k = 0; k < NKIND; ++k) n += (size_t)kind_blocks(c->g, (Kind)k);
        n += (size_t)c->g.ncell;   // moment map of its vector-width class
        size_t tiles = (size_t)((c->g.nx + 3) / 4) * ((c->g.ny + 3) / 4) * c->g.nz;
        n += tiles * 8 * (size_t)sweep_nvb(c->g, 64);
    }
    return n;
}

size_t batch_layout(gsis_batch *b, char *base)
{
    const size_t nc = b->cs.size();
    size_t off = 0;
    carve(off, b->dcases, nc, base);
    carve(off, b->dmap, b->map_cap, base);
    carve(off, b->hist, (size_t)b->hist_cap * nc * 6, base);
    carve(off, b->hist_ctr, 64, base);
    b->case_off.assign(nc, 0);
    for (size_t c = 0; c < nc; ++c) {
        off = align256(off);
        b->case_off[c] = off;
        Dev save = b->cs[c]->d;
        Case *dsave = b->cs[c]->dcase;
        off += layout(b->cs[c], nullptr);
        b->cs[c]->d = save;
        b->cs[c]->dcase = dsave;
    }
    return align256(off);
}

// Case table (with the batch's residual history) to the device.
hipError_t batch_upload_cases(gsis_batch *b)
{
    const int nc = (int)b->cs.size();
    b->hcases.resize(nc);
    for (int c = 0; c < nc; ++c) {
        Case h = b->cs[c]->hcase;
        h.d.hist = b->hist;
        h.d.hist_ctr = b->hist_ctr;
        h.d.hist_index = c;
        h.d.hist_ncase = nc;
        h.d.hist_cap = b->hist_cap;
        b->hcases[c] = h;
    }
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = hipMemcpy(b->dcases, b->hcases.data(), nc * sizeof(Case), hipMemcpyHostToDevice);
    return e;
}

// (case, block) tables of every launch kind and every global sweep plane.
hipError_t batch_build_maps(gsis_batch *b)
{
    const int nc = (int)b->cs.size();
    std::vector<int2> &m = b->hmap;
    m.clear();
    size_t koff[NKIND];
    Target &t = b->t;
    t = Target();
    for (int k = 0; k < NKIND; ++k) {
        koff[k] = m.size();
        for (int c = 0; c < nc; ++c) {
            const int nb = kind_blocks(b->cs[c]->g, (Kind)k);
            for (int j = 0; j < nb; ++j) m.push_back(make_int2(c, j));
        }
        t.nblk[k] = (int)(m.size() - koff[k]);
    }
    size_t moff[3];
    int mcnt[3];
    for (int w = 0; w < 3; ++w) {
        moff[w] = m.size();
        for (int c = 0; c < nc; ++c) {
            if (vw_class(b->cs[c]->vw) != w) continue;
            for (int j = 0; j < b->cs[c]->g.ncell; ++j) m.push_back(make_int2(c, j));
        }
        mcnt[w] = (int)(m.size() - moff[w]);
    }
    int nplane = 0;
    for (const gsis_ctx *c : b->cs) nplane = std::max(nplane, (int)c->plane_cnt.size());
    std::vector<size_t> poff(nplane);
    b->npblk.assign(nplane, 0);
    for (int p = 0; p < nplane; ++p) {
        poff[p] = m.size();
        for (int c = 0; c < nc; ++c) {
            const gsis_ctx *x = b->cs[c];
            if (p >= (int)x->plane_cnt.size()) continue;
            const int nb = x->npblk[p];
            for (int j = 0; j < nb; ++j) m.push_back(make_int2(c, j));
        }
        b->npblk[p] = (int)(m.size() - poff[p]);
    }
    if (m.size() > b->map_cap) return hipErrorInvalidValue;
    for (int k = 0; k < NKIND; ++k) t.map[k] = b->dmap + koff[k];
    for (int w = 0; w < 3; ++w) {
        t.mom_map[w] = b->dmap + moff[w];
        t.mom_nblk[w] = mcnt[w];
    }
    b->pmap.assign(nplane, nullptr);
    for (int p = 0; p < nplane; ++p) b->pmap[p] = b->dmap + poff[p];
    t.cases = b->dcases;
    t.ncase = nc;
    t.host = b->hcases.data();
    t.pmap = b->pmap.data();
    t.npblk = b->npblk.data();
    t.nplane = nplane;
    t.fp32 = b->fp32;
    t.dia = b->dia;
    t.mask = false;
    for (const gsis_ctx *c : b->cs) t.mask = t.mask || c->g.nfluid != c->g.ncell;
    for (const gsis_ctx *c : b->cs) t.g13 = t.g13 || c->g.wall_flux == GSIS_WALLFLUX_G13;
    t.rfn = false;
    t.tx = b->tx;
    t.ty = b->ty;
    t.bs = b->bs;
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess && !m.empty()) e = hipMemcpy(b->dmap, m.data(), m.size() * sizeof(int2), hipMemcpyHostToDevice);
    return e;
}

// One tile shape on every case, then the tables that depend on it.
gsis_status batch_apply_tile(gsis_batch *b, int tx, int ty, int tz, int bs)
{
    for (gsis_ctx *c : b->cs) {
        gsis_status st = gsis_set_tile(c, tx, ty, tz, bs);
        if (st) return bfail(b, st, std::string("tile: ") + c->err);
    }
    const gsis_ctx *c0 = b->cs[0];
    b->tx = c0->tx; b->ty = c0->ty; b->tz = c0->tz; b->bs = c0->bs;
    b->drop_graph();
    if (b->bound) {
        BHIPCHK(b, batch_upload_cases(b));
        BHIPCHK(b, batch_build_maps(b));
    }
    return GSIS_OK;
}

// One GSIS iteration of every case, enqueued on the batch stream.
hipError_t batch_enqueue_iteration(gsis_batch *b, int inner)
{
    const Target &t = b->t;
    hipStream_t s = b->stream;
    hipError_t e = launch_params(t, s);
    if (e == hipSuccess) e = launch_face_scale(t, s);
    if (e == hipSuccess) e = launch_sweep(t, s);
    if (e == hipSuccess) e = launch_moments(t, s);
    if (e == hipSuccess) e = launch_derive(t, s);
    if (inner > 0) {
        if (e == hipSuccess) e = launch_gsis_macro(t, inner, s);
        if (e == hipSuccess) e = launch_commit_correction(t, s);
        if (e == hipSuccess) e = launch_derive(t, s);
    }
    if (e == hipSuccess) e = launch_residual(t, s);
    if (e == hipSuccess) e = launch_snapshot(t, s);
    if (e == hipSuccess) e = launch_hist_advance(b->hist_ctr, s);
    return e;
}

}  // namespace

extern "C" {

const char *gsis_batch_last_error(const gsis_batch *b)
{
    return b ? b->err.c_str() : "no batch";
}

gsis_status gsis_batch_create(gsis_batch **out, gsis_ctx *const *cases, int ncases)
{
    if (!out) return GSIS_EINVAL;
    *out = nullptr;
    if (!cases || ncases < 1 || ncases > 4096) return GSIS_EINVAL;
    for (int i = 0; i < ncases; ++i) {
        gsis_ctx *c = cases[i];
        if (!c || c->bound) return GSIS_EINVAL;
        for (int j = 0; j < i; ++j)
            if (cases[j] == c) return GSIS_EINVAL;
        if (c->fp32 != cases[0]->fp32 || c->g.species != cases[0]->g.species) return GSIS_EINVAL;
        if (c->g.inv_dt != 0.0 || c->g.order != 1 || c->g.vlist || c->g.umesh) return GSIS_EINVAL;
    }
    gsis_batch *b = new (std::nothrow) gsis_batch();
    if (!b) return GSIS_ENOMEM;
    b->cs.assign(cases, cases + ncases);
    b->fp32 = cases[0]->fp32;
    b->dia = cases[0]->g.species == GSIS_DIATOMIC;
    gsis_status st = batch_apply_tile(b, 0, 0, 0, 0);
    if (st) {
        delete b;
        return st;
    }
    for (gsis_ctx *c : b->cs)
        if (!c->meta_ready) build_meta(c);
    b->map_cap = batch_map_cap(b);
    *out = b;
    return GSIS_OK;
}

gsis_status gsis_batch_destroy(gsis_batch *b)
{
    if (!b) return GSIS_EINVAL;
    delete b;
    return GSIS_OK;
}

gsis_status gsis_batch_workspace_size(gsis_batch *b, size_t *bytes)
{
    if (!b || !bytes) return GSIS_EINVAL;
    Case *dc = b->dcases;
    int2 *dm = b->dmap;
    double *h = b->hist;
    int *hc = b->hist_ctr;
    *bytes = batch_layout(b, nullptr);
    b->dcases = dc; b->dmap = dm; b->hist = h; b->hist_ctr = hc;
    return GSIS_OK;
}

gsis_status gsis_batch_bind_workspace(gsis_batch *b, void *device_ptr, size_t bytes)
{
    if (!b) return GSIS_EINVAL;
    if (b->bound) return bfail(b, GSIS_ESTATE, "workspace already bound");
    if (!device_ptr) return bfail(b, GSIS_EINVAL, "workspace pointer is NULL");
    if ((uintptr_t)device_ptr % 256) return bfail(b, GSIS_EINVAL, "workspace must be 256-byte aligned");
    size_t need;
    gsis_batch_workspace_size(b, &need);
    if (bytes < need) return bfail(b, GSIS_ENOMEM, "workspace smaller than gsis_batch_workspace_size");
    char *base = (char *)device_ptr;
    batch_layout(b, base);
    for (size_t c = 0; c < b->cs.size(); ++c) {
        gsis_ctx *x = b->cs[c];
        size_t sz = 0;
        gsis_workspace_size(x, &sz);
        gsis_status st = gsis_bind_workspace(x, base + b->case_off[c], sz);
        if (st) return bfail(b, st, "case " + std::to_string(c) + ": " + x->err);
        x->stream = b->stream;
    }
    b->ws = base;
    b->ws_bytes = bytes;
    BHIPCHK(b, hipMemset(b->hist_ctr, 0, 64 * sizeof(int)));
    BHIPCHK(b, batch_upload_cases(b));
    BHIPCHK(b, batch_build_maps(b));
    BHIPCHK(b, hipDeviceSynchronize());
    b->bound = true;
    return GSIS_OK;
}

gsis_status gsis_batch_set_stream(gsis_batch *b, void *hip_stream)
{
    if (!b) return GSIS_EINVAL;
    b->stream = (hipStream_t)hip_stream;
    for (gsis_ctx *c : b->cs) c->stream = b->stream;
    return GSIS_OK;
}

gsis_status gsis_batch_set_tile(gsis_batch *b, int tx, int ty, int tz, int block)
{
    if (!b) return GSIS_EINVAL;
    return batch_apply_tile(b, tx, ty, tz, block);
}

gsis_status gsis_batch_get_tile(const gsis_batch *b, int *tile)
{
    if (!b || !tile) return GSIS_EINVAL;
    tile[0] = b->tx; tile[1] = b->ty; tile[2] = b->tz; tile[3] = b->bs;
    return GSIS_OK;
}

gsis_status gsis_batch_init_maxwellian(gsis_batch *b, double rho, const double u[3], double T, double Tr)
{
    if (!b) return GSIS_EINVAL;
    if (!b->bound) return bfail(b, GSIS_ESTATE, "bind_workspace first");
    for (size_t c = 0; c < b->cs.size(); ++c) {
        gsis_status st = gsis_init_maxwellian(b->cs[c], rho, u, T, Tr);
        if (st) return bfail(b, st, "case " + std::to_string(c) + ": " + b->cs[c]->err);
    }
    BHIPCHK(b, launch_zero_int(b->hist_ctr, 1, b->stream));
    b->iters_run = 0;
    b->inited = true;
    return GSIS_OK;
}

gsis_status gsis_batch_autotune(gsis_batch *b, int reps, int *cfg_out, double *ms_out, int max, int *count)
{
    if (!b) return GSIS_EINVAL;
    if (!b->inited) return bfail(b, GSIS_ESTATE, "initialise the batch first");
    if (reps < 1 || max < 0) return bfail(b, GSIS_EINVAL, "reps must be >= 1");
    const gsis_ctx *c0 = b->cs[0];
    int shapes[32];
    int nsh = sweep_shapes(b->fp32, shapes, 16);
    struct Cand { int tx, ty, tz, bs; double ms; };
    std::vector<Cand> cands;
    for (int k = 0; k < nsh; ++k) {
        int tx = shapes[2 * k], ty = shapes[2 * k + 1];
        if (!sweep_shape_supported(b->fp32, b->dia, tx, ty)) continue;
        const int nw = sweep_shape_waves(b->fp32, tx, ty);
        for (int tz : {tx / 2, tx, 2 * tx, 4 * tx})
            for (int bs : {64, 128, 256})
                if (nw == 1 || bs == 64 * nw) cands.push_back({tx, ty, std::max(tz, 1), bs, 0.0});
    }
    (void)c0;
    const int save[4] = {b->tx, b->ty, b->tz, b->bs};
    BHIPCHK(b, launch_params(b->t, b->stream));
    BHIPCHK(b, launch_face_scale(b->t, b->stream));
    hipEvent_t e0, e1;
    BHIPCHK(b, hipEventCreate(&e0));
    BHIPCHK(b, hipEventCreate(&e1));
    gsis_status st = GSIS_OK;
    for (auto &c : cands) {
        st = batch_apply_tile(b, c.tx, c.ty, c.tz, c.bs);
        if (st) break;
        hipError_t e = launch_sweep(b->t, b->stream);   // warm-up launch of this configuration
        if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_sweep(b->t, b->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) { st = bfail(b, GSIS_EDEVICE, std::string("autotune: ") + hipGetErrorString(e)); break; }
        c.ms = ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) {
        batch_apply_tile(b, save[0], save[1], save[2], save[3]);
        return st;
    }
    size_t best = 0;
    for (size_t k = 1; k < cands.size(); ++k)
        if (cands[k].ms < cands[best].ms) best = k;
    st = batch_apply_tile(b, cands[best].tx, cands[best].ty, cands[best].tz, cands[best].bs);
    if (st) return st;
    // every case now holds this pass's sweep result (identical under every configuration)
    BHIPCHK(b, launch_moments(b->t, b->stream));
    BHIPCHK(b, launch_derive(b->t, b->stream));
    for (gsis_ctx *c : b->cs) {
        c->pending = false;
        c->passes++;
        c->stepped = true;
    }
    int n = 0;
    for (size_t k = 0; k < cands.size() && n < max; ++k, ++n) {
        if (cfg_out) {
            cfg_out[4 * n] = cands[k].tx; cfg_out[4 * n + 1] = cands[k].ty;
            cfg_out[4 * n + 2] = cands[k].tz; cfg_out[4 * n + 3] = cands[k].bs;
        }
        if (ms_out) ms_out[n] = cands[k].ms;
    }
    if (count) *count = n;
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    return GSIS_OK;
}

gsis_status gsis_batch_run(gsis_batch *b, int iters, int inner_iters, int use_graph)
{
    if (!b) return GSIS_EINVAL;
    if (!b->inited) return bfail(b, GSIS_ESTATE, "initialise the batch first");
    if (iters < 0 || inner_iters < 0) return bfail(b, GSIS_EINVAL, "iters and inner_iters must be >= 0");
    if (use_graph && !b->stream) return bfail(b, GSIS_EINVAL, "graph capture needs a non-null stream");
    for (gsis_ctx *c : b->cs)
        if (!c->inited) return bfail(b, GSIS_ESTATE, "a case was not initialised");
    if (!b->ev0) BHIPCHK(b, hipEventCreate(&b->ev0));
    if (!b->ev1) BHIPCHK(b, hipEventCreate(&b->ev1));
    if (use_graph && iters > 0 && (!b->exec || b->graph_inner != inner_iters)) {
        b->drop_graph();
        BHIPCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = batch_enqueue_iteration(b, inner_iters);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return bfail(b, GSIS_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
        }
        b->graph = g;
        BHIPCHK(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->graph_inner = inner_iters;
    }
    BHIPCHK(b, hipEventRecord(b->ev0, b->stream));
    for (int it = 0; it < iters; ++it) {
        if (use_graph) BHIPCHK(b, hipGraphLaunch(b->exec, b->stream));
        else BHIPCHK(b, batch_enqueue_iteration(b, inner_iters));
    }
    BHIPCHK(b, hipEventRecord(b->ev1, b->stream));
    b->timed = true;
    for (gsis_ctx *c : b->cs) {
        c->passes += iters;
        if (iters > 0) {
            c->stepped = true;
            c->pending = inner_iters > 0;
        }
    }
    b->iters_run += iters;
    return GSIS_OK;
}

gsis_status gsis_batch_residuals(gsis_batch *b, double *eps, int max, int *count)
{
    if (!b || !count || max < 0) return GSIS_EINVAL;
    if (!b->bound) return bfail(b, GSIS_ESTATE, "bind_workspace first");
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    const int nc = (int)b->cs.size();
    int ctr = 0;
    BHIPCHK(b, hipMemcpy(&ctr, b->hist_ctr, sizeof(int), hipMemcpyDeviceToHost));
    int n = std::min(std::min(ctr, b->hist_cap), max);
    std::vector<double> h((size_t)b->hist_cap * nc * 6);
    BHIPCHK(b, hipMemcpy(h.data(), b->hist, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int i = 0; i < n && eps; ++i) {
        const int slot = (ctr - n + i) % b->hist_cap;
        for (int c = 0; c < nc; ++c) {
            const double *v = &h[((size_t)slot * nc + c) * 6];
            const ResidEval r = resid_eval(v, b->cs[c]->fp32);
            for (int k = 0; k < 3; ++k) eps[((size_t)i * nc + c) * 3 + k] = r.eps[k];
        }
    }
    *count = n;
    for (int c = 0; c < nc; ++c) {
        int flag = 0;
        BHIPCHK(b, hipMemcpy(&flag, b->cs[c]->d.errflag, sizeof(int), hipMemcpyDeviceToHost));
        if (flag) return bfail(b, GSIS_ENOTFINITE, "case " + std::to_string(c) + " flagged a non-physical state (" +
                                                         std::to_string(flag) + ")");
    }
    return GSIS_OK;
}

gsis_status gsis_batch_last_run_ms(gsis_batch *b, double *ms)
{
    if (!b || !ms) return GSIS_EINVAL;
    if (!b->timed) return bfail(b, GSIS_ESTATE, "no run yet");
    BHIPCHK(b, hipEventSynchronize(b->ev1));
    float t = 0.0f;
    BHIPCHK(b, hipEventElapsedTime(&t, b->ev0, b->ev1));
    *ms = t;
    return GSIS_OK;
}

}  // extern "C"

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
// registers one slab ahead; the VDF stores and the inflow-face reads are
// non-temporal (streamed past the caches: nothing reads them back soon).
// The reference distribution is evaluated on the
// fly from the per-cell parameters (FP32 copies on the FP32 path), one
// exponential per Maxwellian shape.  Every cell's update has a fixed operand
// order, so the result is bitwise independent of the tile shape and of the
// schedule.
#include "gsis_common.h"
#include "gsis_launch.h"
#include "gsis_sweep_math.h"

namespace gsis {

// TX x TY is the slab one wave holds.  With a wave grid (WX x WY > 1) a
// block of WX WY waves owns a (WX TX) x (WY TY) tile for one run of 64 nodes:
// wave (wx, wy) holds sub-tile (wx, wy) and runs WX + WY - 2 steps behind
// (wx + wy steps after the first), so at every step the slab it works on has
// its x- and y-upwind slabs finished by the waves before it, which hand over
// their exit faces through LDS (double buffered by step parity, one barrier
// per step).  Only the tile's own inflow faces are read from the VDF, so a
// wave grid reads 1/(WX TX) + 1/(WY TY) + 1/TZ of the points again instead of
// 1/TX + 1/TY + 1/TZ.
// eoff >= 0: the launch covers the plane's (tile, octant) entries from eoff
// on (a split sweep: clean entries in the kernel without the solid-cell
// logic, the rest in the masked one); eoff < 0: every tile of the plane for
// all 8 octants.
//
// Occupancy: the FP64 monatomic 4 x 4 slab is held to 168 VGPRs, three waves
// per SIMD (measured 5-7% faster than two waves without the few spills this
// costs); the other shapes take what they need.
template <typename T, int TX, int TY, int WX, int WY, bool DIA, bool RFN, bool MASK>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu((sizeof(T) == 8 && TX * TY == 16 && !DIA) ? 3 : 1)))
void k_sweep(GSIS_SPAN_ARGS, int plane, int eoff)
{
    // no automatic contraction: every fused multiply-add is written out, so the
    // operations of a cell update do not depend on the surrounding code
#pragma clang fp contract(off)
    constexpr int NWV = WX * WY;                  // waves sharing the nodes of a block
    constexpr bool GRID = NWV > 1;
    constexpr int NPL = DIA ? 36 : 16;            // parameters per cell kept in LDS
    // the last two LDS slots of a cell (unused by the parameters) carry the
    // density scales of its x- and y-upwind faces, for the tile's inflow faces
    constexpr int SXS = NPL - 2, SYS = NPL - 1;
    constexpr int NC = TX * TY;                   // cells per slab
    constexpr int NM = NC * NPL;                  // parameter words per slab
    constexpr int MPT = (NM + 63) / 64;           // words per thread for the smallest block (64)
    __shared__ T spar[NWV][2][NM];
    __shared__ int sflag[NWV][2][NC];
    // exit faces handed downstream inside a wave grid: x faces written by the
    // waves with wx < WX - 1, y faces by those with wy < WY - 1
    constexpr int ND = DIA ? 2 : 1;
    constexpr int XWN = GRID && WX > 1 ? (WX - 1) * WY : 1, YWN = GRID && WY > 1 ? WX * (WY - 1) : 1;
    constexpr int FXN = GRID ? TY : 1, FYN = GRID ? TX : 1, FL = GRID ? 64 : 1;
    __shared__ T xface[ND][XWN][2][FXN][FL];
    __shared__ T yface[ND][YWN][2][FYN][FL];

    int b;
    const Case &C = case_of(span_cases, span_map, b);
    const Geo &g = C.g;
    constexpr bool F32 = sizeof(T) == 4;
    const int TZ = C.tz, nvb = C.nvb;
    const gptr<const int> cflag = (gptr<const int>)C.d.cflag;
    // data every lane reads at the same index (neighbour flags, face scales, the
    // tile lists) go through the scalar unit: the constant address space, as for
    // the case record (none of it changes while the sweep runs)
    const cptr<int> cflags = (cptr<int>)C.d.cflag;
    const int plane_off = ((cptr<int>)C.d.plane_off)[plane];
    const int vb = b % nvb;
    int o, t;
    if (eoff >= 0) {
        const int ent = ((cptr<int>)C.d.tent)[8 * plane_off + eoff + b / nvb];
        o = ent & 7;
        t = ent >> 3;
    } else {
        o = (b / nvb) & 7;
        t = b / (nvb * 8);
    }
    const int lane = threadIdx.x & 63;
    const int w = GRID ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : 0;
    const int wx = w % WX, wy = w / WX;
    const int bs = GRID ? 64 : (int)blockDim.x;   // nodes per block, and threads of the meta loads
    const int ml = GRID ? lane : (int)threadIdx.x;
    if (vb * bs >= g.osize[o]) return;            // a node run past the end of a smaller octant
    const int l = vb * bs + ml;
    const bool active = l < g.osize[o];           // inactive threads still join loads and barriers
    const int packed = ((cptr<int>)C.d.tiles)[plane_off + t];
    const int tx = packed & 0x3ff, ty = (packed >> 10) & 0x3ff, tz = (packed >> 20) & 0x3ff;
    const int sx = o & 1, sy = (o >> 1) & 1, sz = (o >> 2) & 1;
    const int dxu = sx, dyu = 2 + sy, dzu = 4 + sz;   // upwind faces
    // origin of this wave's slab column (the tile's, for a single wave)
    const int i0 = tx * (TX * WX) + wx * TX, j0 = ty * (TY * WY) + wy * TY, k0 = tz * TZ;
    const int nx = g.nx, ny = g.ny, nz = g.nz, ncell = g.ncell;
    const size_t nv = (size_t)g.nv;

    T xix = T(0), xiy = T(0), xiz = T(0);
    size_t node = 0;
    if (active) {
        node = (size_t)g.obase[o] + l;
        const gptr<const T> nt = (F32 ? (gptr<const T>)C.d.nt32 : (gptr<const T>)C.d.nt64) + 4 * node;
        xix = nt[0];
        xiy = nt[1];
        xiz = nt[2];
    }
    const T ax = fabs(xix) * (T)g.invh[0];
    const T ay = fabs(xiy) * (T)g.invh[1];
    const T az = fabs(xiz) * (T)g.invh[2];
    const T idt = (T)g.inv_dt;
    const T den0 = idt + ax + ay + az;
    const gptr<T> f0 = (gptr<T>)C.d.f0;
    const gptr<T> f1 = (gptr<T>)C.d.f1;
    const gptr<const T> rs0 = (gptr<const T>)C.d.rs0;   // per-point term (RFN)
    const gptr<const T> rs1 = (gptr<const T>)C.d.rs1;
    const T rsc = (T)g.rs_scale;
    const gptr<const T> par = F32 ? (gptr<const T>)C.d.parf : (gptr<const T>)C.d.par;
    const cptr<T> fsc = F32 ? (cptr<T>)C.d.cfs32 : (cptr<T>)C.d.cfs64;   // [ncell][6] incoming density scale
    const gptr<const T> fscv = F32 ? (gptr<const T>)C.d.cfs32 : (gptr<const T>)C.d.cfs64;   // the same, per lane
    const gptr<const T> mb = F32 ? (gptr<const T>)C.d.mb32 : (gptr<const T>)C.d.mb64;
    const gptr<const T> mb1 = F32 ? (gptr<const T>)C.d.mb1_32 : (gptr<const T>)C.d.mb1_64;
    // VDF rows by pointer: row r of buffer p starts at p + r nv elements, and a
    // lane adds the 32-bit byte offset of its node (every VDF access is a
    // uniform row address plus this lane offset)
    const size_t rowb = nv * sizeof(T);
    const unsigned loff = (unsigned)node * (unsigned)sizeof(T);
    auto rowp = [&](auto base, int r) -> gptr<char> { return (gptr<char>)base + (size_t)r * rowb; };
    auto lane_at = [&](gptr<char> rp) -> T * { return (T *)(rp + loff); };
    // boundary Maxwellians of this lane's node, for the whole tile: the box
    // faces upwind along x, y, z and the solid surface
    T mbu[3], mbu1[3], mbs = T(0), mbs1 = T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int d = a == 0 ? dxu : (a == 1 ? dyu : dzu);
        mbu[a] = mb[(size_t)d * nv + node];
        mbu1[a] = DIA ? mb1[(size_t)d * nv + node] : T(0);
    }
    if (MASK) {
        mbs = mb[(size_t)6 * nv + node];
        if (DIA) mbs1 = mb1[(size_t)6 * nv + node];
    }

    // physical cell of tile-frame position, clamped into the domain (positions
    // outside are never computed; clamping keeps every speculative load valid)
    auto cell_of = [&](int kx, int ky, int kz) -> int {
        int ii = min(i0 + kx, nx - 1), jj = min(j0 + ky, ny - 1), kk = min(k0 + kz, nz - 1);
        const int i = sx ? nx - 1 - ii : ii, j = sy ? ny - 1 - jj : jj, k = sz ? nz - 1 - kk : kk;
        return i + nx * (j + ny * k);
    };
    auto inside = [&](int kx, int ky, int kz) -> bool { return i0 + kx < nx && j0 + ky < ny && k0 + kz < nz; };
    // Value entering cell c through its upwind face d: the neighbour's f^{n+1/2}
    // (final: the upwind tile ran earlier, the VDF is updated in place) or the
    // boundary value rho_b M_b(xi) of the face.  All loads are independent and
    // unconditional, so they can be issued a slab ahead.
    // With handed (a face inside a wave grid) the neighbour's value arrives in
    // LDS later: only the wall value and flag are prepared here.
    // upwind neighbour of cell c across face d (c itself where the face is on the box)
    auto upwind_of = [&](int c, int kx, int ky, int kz, int d, bool &outside) -> int {
        const int a = d >> 1;
        const int ii = i0 + kx, jj = j0 + ky, kk = k0 + kz;   // tile frame; upwind = one step back
        outside = (a == 0 ? ii : (a == 1 ? jj : kk)) == 0;
        const int step = a == 0 ? 1 : (a == 1 ? nx : nx * ny);
        return outside ? c : ((d & 1) ? c + step : c - step);
    };
    // the neighbour's value across an x or y inflow face of the slab (the wall
    // value of a face on the box or a solid cell is formed where it is used,
    // from the face scale staged with the slab's parameters)
    auto inflow = [&](int c, int kx, int ky, int kz, int d, T &v0, T &v1, bool handed) {
        bool outside;
        const int nb = upwind_of(c, kx, ky, kz, d, outside);
        v0 = handed ? T(0) : __builtin_nontemporal_load(lane_at(rowp(f0, nb)));
        if (DIA) v1 = handed ? T(0) : __builtin_nontemporal_load(lane_at(rowp(f1, nb)));
    };
    // the value entering the tile's first slab through its z face: the
    // neighbour's or the boundary value rho_b M_b(xi) of the face
    auto inflow_z = [&](int c, int kx, int ky, T &v0, T &v1) {
        bool outside;
        const int nb = upwind_of(c, kx, ky, 0, dzu, outside);
        const T fv0 = __builtin_nontemporal_load(lane_at(rowp(f0, nb)));
        const T sc = fsc[(size_t)c * 6 + dzu];
        const bool wall = outside || (MASK && !cflags[nb]);
        v0 = wall ? sc * (outside ? mbu[2] : mbs) : fv0;
        if (DIA) {
            const T fv1 = __builtin_nontemporal_load(lane_at(rowp(f1, nb)));
            v1 = wall ? sc * (outside ? mbu1[2] : mbs1) : fv1;
        }
    };
    // boundary value of face d of cell c when the in-tile upwind cell is solid
    auto solid_face = [&](int c, int d, T &v0, T &v1) {
        const T sc = fsc[(size_t)c * 6 + d];
        v0 = sc * mbs;
        if (DIA) v1 = sc * mbs1;
    };

    T mreg[MPT];
    int freg = 0;
    auto issue_meta = [&](int kz) {
#pragma unroll
        for (int r = 0; r < MPT; ++r) {
            if (r * bs >= NM) break;                      // uniform: larger blocks need fewer rounds
            const int e = min(ml + r * bs, NM - 1);
            const int cc = e / NPL, k = e % NPL;
            const int c = cell_of(cc % TX, cc / TX, kz);
            mreg[r] = k < SXS ? par[(size_t)c * NPAR + k] : fscv[(size_t)c * 6 + (k == SXS ? dxu : dyu)];
        }
        // flag word of a cell: bit 0 fluid and inside the domain, bit 1 its in-tile
        // z-upwind cell is solid, bits 2 and 3 the cell of the previous column
        // (row) that sends the slab's x (y) inflow is solid (carried with this
        // slab so that compute never reads the other buffer, which the next
        // slab's data may be overwriting)
        const int e = min(ml, NC - 1);
        const int c = cell_of(e % TX, e / TX, kz);
        const int cz = cell_of(e % TX, e / TX, kz > 0 ? kz - 1 : 0);
        const int fl = (MASK ? cflag[c] : 1) && inside(e % TX, e / TX, kz);
        const int zs = (MASK && kz > 0) ? !cflag[cz] : 0;
        const int xs = (MASK && e % TX == 0 && i0 > 0) ? !cflag[sx ? c + 1 : c - 1] : 0;
        const int ys = (MASK && e / TX == 0 && j0 > 0) ? !cflag[sy ? c + nx : c - nx] : 0;
        freg = fl | (zs << 1) | (xs << 2) | (ys << 3);
    };
    auto store_meta = [&](int buf) {
#pragma unroll
        for (int r = 0; r < MPT; ++r) {
            if (r * bs >= NM) break;
            const int e = ml + r * bs;
            if (e < NM) spar[w][buf][e] = mreg[r];
        }
        if (ml < NC) sflag[w][buf][ml] = freg;
    };

    T pl0[TY][TX], pl1[TY][TX];                 // z-upwind plane, then the slab just computed
    T xin0[TY], xin1[TY], yin0[TX], yin1[TX];   // inflow faces of the current slab
    T xnx0[TY], xnx1[TY], ynx0[TX], ynx1[TX];   // ... and of the next slab
    const bool xhand = GRID && wx > 0, yhand = GRID && wy > 0;   // uniform per wave
    const bool xbox = i0 == 0, ybox = j0 == 0;  // the slab column's x (y) inflow face is on the box
    auto issue_xy = [&](int kz, T *x0, T *x1, T *y0, T *y1) {
#pragma unroll
        for (int ky = 0; ky < TY; ++ky) inflow(cell_of(0, ky, kz), 0, ky, kz, dxu, x0[ky], x1[ky], xhand);
#pragma unroll
        for (int kx = 0; kx < TX; ++kx) inflow(cell_of(kx, 0, kz), kx, 0, kz, dyu, y0[kx], y1[kx], yhand);
    };

    issue_meta(0);
    store_meta(0);
#pragma unroll
    for (int ky = 0; ky < TY; ++ky)
#pragma unroll
        for (int kx = 0; kx < TX; ++kx) inflow_z(cell_of(kx, ky, 0), kx, ky, pl0[ky][kx], pl1[ky][kx]);
    issue_xy(0, xin0, xin1, yin0, yin1);
    __syncthreads();

    // per-tile strides of the octant frame: cell = slab base + kx dxs + ky dys
    const int dxs = sx ? -1 : 1, dys = sy ? -nx : nx;
    // slabs of this tile and steps of the block (uniform over the block)
    const int TZe = max(0, min(TZ, nz - k0));
    const int nstep = TZe + (WX - 1) + (WY - 1);
    const int xr = wy * (WX - 1) + wx - 1, xw = wy * (WX - 1) + wx;   // x-face slots read / written
    const int yr = (wy - 1) * WX + wx, yw = wy * WX + wx;             // y-face slots read / written
    for (int st = 0; st < nstep; ++st) {
        const int kz = st - (wx + wy);            // the slab of this wave at this step
        const bool run = kz >= 0 && kz < TZe;     // uniform over the wave
        const int buf = kz & 1;
        const bool more = run && kz + 1 < TZe;
        if (more) {
            issue_meta(kz + 1);
            issue_xy(kz + 1, xnx0, xnx1, ynx0, ynx1);
        }
        const int kk = k0 + kz;
        const int cbase = (sx ? nx - 1 - i0 : i0) + nx * ((sy ? ny - 1 - j0 : j0) + ny * (sz ? nz - 1 - kk : kk));
        // cell (kx, ky) of the slab is row cbase + kx dxs + ky dys; its row pointer
        // is the slab's plus constant strides (a dead cell's is the sink row's)
        const ptrdiff_t sxb = (ptrdiff_t)dxs * (ptrdiff_t)rowb, syb = (ptrdiff_t)dys * (ptrdiff_t)rowb;
        auto cellp = [&](auto base, int kx, int ky, bool live) -> gptr<char> {
            return live ? rowp(base, cbase) + ((ptrdiff_t)kx * sxb + (ptrdiff_t)ky * syb) : rowp(base, ncell);
        };
        if (GRID && run) {
            // exit faces of the upwind waves' slab kz, written at the previous step
            const int pb = (st - 1) & 1;
            if (xhand) {
#pragma unroll
                for (int ky = 0; ky < TY; ++ky) {
                    xin0[ky] = xface[0][xr][pb][ky][lane];
                    if (DIA) xin1[ky] = xface[ND - 1][xr][pb][ky][lane];
                }
            }
            if (yhand) {
#pragma unroll
                for (int kx = 0; kx < TX; ++kx) {
                    yin0[kx] = yface[0][yr][pb][kx][lane];
                    if (DIA) yin1[kx] = yface[ND - 1][yr][pb][kx][lane];
                }
            }
        }
        if (run && active) {
            // The per-point term of every cell of the slab (RFN), read before
            // the slab's first store: a read placed at its cell would wait for
            // the stores before it (the two buffers may alias as far as the
            // compiler knows), one load latency per cell.  Not for the FP64
            // diatomic masked 8 x 4 slab, whose registers are already full
            // (the held terms spilled to scratch); it reads at the cell.
            constexpr bool HOIST = RFN && !(DIA && MASK && !F32 && TX * TY > 16);
            T rv0[HOIST ? TY : 1][HOIST ? TX : 1], rv1[HOIST && DIA ? TY : 1][HOIST && DIA ? TX : 1];
            if constexpr (HOIST) {
#pragma unroll
                for (int ky = 0; ky < TY; ++ky) {
#pragma unroll
                    for (int kx = 0; kx < TX; ++kx) {
                        const int e = ky * TX + kx;
                        const int flag = MASK ? __builtin_amdgcn_readfirstlane(sflag[w][buf][e]) : 1;
                        const bool live = MASK ? (flag & 1) != 0 : (i0 + kx < nx && j0 + ky < ny);
                        rv0[ky][kx] = __builtin_nontemporal_load(lane_at(cellp(rs0, kx, ky, live)));
                        if (DIA) rv1[ky][kx] = __builtin_nontemporal_load(lane_at(cellp(rs1, kx, ky, live)));
                    }
                }
            }
            // Monatomic gas without solid cells: the parameters that start a
            // cell's exponential (u and 1/T) are read from LDS one cell ahead and
            // the rest before the exponential, held there by a scheduling
            // barrier (measured: slower with the per-cell branches of solid
            // cells and with the diatomic gas's larger register planes).
            constexpr bool PRE = !MASK && !DIA;
            constexpr int NPRE = 4;
            T pre[NPRE];
            if (PRE) {
#pragma unroll
                for (int k = 0; k < NPRE; ++k) pre[k] = spar[w][buf][k];
            }
#pragma unroll
            for (int ky = 0; ky < TY; ++ky) {
#pragma unroll
                for (int kx = 0; kx < TX; ++kx) {
                    const int e = ky * TX + kx;
                    T cur[NPRE], rest[NPL];
                    if constexpr (PRE) {
#pragma unroll
                        for (int k = 0; k < NPRE; ++k) cur[k] = pre[k];
                        if (e + 1 < NC) {
#pragma unroll
                            for (int k = 0; k < NPRE; ++k) pre[k] = spar[w][buf][(e + 1) * NPL + k];
                        }
#pragma unroll
                        for (int k = NPRE; k < 14; ++k) rest[k] = spar[w][buf][e * NPL + k];
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    // Every cell of the slab is computed, so the slab is straight-line
                    // code; a cell outside the domain or solid stores into the sink row
                    // (row ncell) and its value is never used upwind.
                    const int flag = MASK ? __builtin_amdgcn_readfirstlane(sflag[w][buf][e]) : 1;
                    const bool live = MASK ? (flag & 1) != 0 : (i0 + kx < nx && j0 + ky < ny);
                    const int cell = cbase + kx * dxs + ky * dys;
                    const int cread = live ? cell : 0;   // in-range index for side reads
                    const gptr<char> c0 = cellp(f0, kx, ky, live);   // uniform row; the lane adds its node
                    const gptr<char> c1 = DIA ? cellp(f1, kx, ky, live) : c0;
                    const T *p = PRE ? rest : &spar[w][buf][e * NPL];
                    const T cx = xix - (PRE ? cur[0] : p[0]), cy = xiy - (PRE ? cur[1] : p[1]), cz = xiz - (PRE ? cur[2] : p[2]);
                    T gt0, gt1 = T(0), invtau;
                    if (DIA) {
                        ref_dia<T>(p, cx, cy, cz, p[3], p[4], gt0, gt1);
                        invtau = p[33];
                    } else {
                        gt0 = ref_mono<T>(p, cx, cy, cz, PRE ? cur[3] : p[3]);
                        invtau = p[13];
                    }
                    T num0 = gt0, num1 = gt1;
                    if constexpr (HOIST) {
                        num0 = fma(rsc, rv0[ky][kx], num0);
                        if (DIA) num1 = fma(rsc, rv1[ky][DIA ? kx : 0], num1);
                    } else if constexpr (RFN) {
                        num0 = fma(rsc, __builtin_nontemporal_load(lane_at(cellp(rs0, kx, ky, live))), num0);
                        if (DIA) num1 = fma(rsc, __builtin_nontemporal_load(lane_at(cellp(rs1, kx, ky, live))), num1);
                    }
                    T F0, F1 = T(0);
                    if (kx == 0) {
                        if (xbox || (MASK && (flag & 4))) {   // a wall: the box face or a solid cell
                            const T sc = spar[w][buf][e * NPL + SXS];
                            F0 = sc * (xbox ? mbu[0] : mbs);
                            if (DIA) F1 = sc * (xbox ? mbu1[0] : mbs1);
                        } else { F0 = xin0[ky]; if (DIA) F1 = xin1[ky]; }
                    }
                    else if (MASK && !(__builtin_amdgcn_readfirstlane(sflag[w][buf][e - 1]) & 1)) solid_face(cread, dxu, F0, F1);
                    else { F0 = pl0[ky][kx - 1]; if (DIA) F1 = pl1[ky][kx - 1]; }
                    num0 = fma(ax, F0, num0);
                    if (DIA) num1 = fma(ax, F1, num1);
                    if (ky == 0) {
                        if (ybox || (MASK && (flag & 8))) {
                            const T sc = spar[w][buf][e * NPL + SYS];
                            F0 = sc * (ybox ? mbu[1] : mbs);
                            if (DIA) F1 = sc * (ybox ? mbu1[1] : mbs1);
                        } else { F0 = yin0[kx]; if (DIA) F1 = yin1[kx]; }
                    }
                    else if (MASK && !(__builtin_amdgcn_readfirstlane(sflag[w][buf][e - TX]) & 1)) solid_face(cread, dyu, F0, F1);
                    else { F0 = pl0[ky - 1][kx]; if (DIA) F1 = pl1[ky - 1][kx]; }
                    num0 = fma(ay, F0, num0);
                    if (DIA) num1 = fma(ay, F1, num1);
                    if (MASK && (flag & 2)) solid_face(cread, dzu, F0, F1);
                    else { F0 = pl0[ky][kx]; if (DIA) F1 = pl1[ky][kx]; }
                    num0 = fma(az, F0, num0);
                    if (DIA) num1 = fma(az, F1, num1);
                    const T den = den0 + invtau;
                    const T v0 = Arith<T>::div(num0, den);
                    __builtin_nontemporal_store(v0, lane_at(c0));
                    pl0[ky][kx] = v0;
                    if (DIA) {
                        const T v1 = Arith<T>::div(num1, den);
                        __builtin_nontemporal_store(v1, lane_at(c1));
                        pl1[ky][kx] = v1;
                    }
                }
            }
        }
        if (GRID && run) {
            // this slab's exit faces for the downstream waves (every lane, so the
            // reads of inactive lanes stay defined)
            if (WX > 1 && wx < WX - 1) {
#pragma unroll
                for (int ky = 0; ky < TY; ++ky) {
                    xface[0][xw][st & 1][ky][lane] = pl0[ky][TX - 1];
                    if (DIA) xface[ND - 1][xw][st & 1][ky][lane] = pl1[ky][TX - 1];
                }
            }
            if (WY > 1 && wy < WY - 1) {
#pragma unroll
                for (int kx = 0; kx < TX; ++kx) {
                    yface[0][yw][st & 1][kx][lane] = pl0[TY - 1][kx];
                    if (DIA) yface[ND - 1][yw][st & 1][kx][lane] = pl1[TY - 1][kx];
                }
            }
        }
        if (more) store_meta(buf ^ 1);
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
// A tile shape (tx, ty) is served by slabs of (tx / wx) x (ty / wy) cells held
// by a wx x wy wave grid (one wave: wx = wy = 1).  tz is a run-time loop
// length.  The slab is held in registers, so the diatomic gas (two planes)
// uses slabs of at most 32 cells.
struct Shape { int tx, ty, wx, wy; };
static const Shape kShapes32[] = {{4, 4, 1, 1}, {8, 4, 1, 1}, {8, 8, 1, 1}, {16, 8, 2, 2}};
static const Shape kShapes64[] = {{4, 4, 1, 1}, {8, 4, 1, 1}, {8, 8, 2, 2}};

static const Shape *find_shape(bool fp32, int tx, int ty)
{
    const Shape *sh = fp32 ? kShapes32 : kShapes64;
    const int cnt = fp32 ? (int)(sizeof(kShapes32) / sizeof(Shape)) : (int)(sizeof(kShapes64) / sizeof(Shape));
    for (int k = 0; k < cnt; ++k)
        if (sh[k].tx == tx && sh[k].ty == ty) return &sh[k];
    return nullptr;
}

template <typename T, int TX, int TY, int WX, int WY>
static void sweep_launch(const Target &t, int p, hipStream_t s, unsigned nblk, bool mask, int eoff)
{
    constexpr bool kDia = TX * TY <= 32;   // two register planes only for the small slabs
    const dim3 grid(nblk);
    const Span sp{t.cases, t.pmap ? t.pmap[p] : nullptr};
#define GSIS_SWEEP(D, R, M) \
    hipLaunchKernelGGL((k_sweep<T, TX, TY, WX, WY, D, R, M>), grid, dim3(t.bs), 0, s, GSIS_SPAN(sp), p, eoff)
    if (t.dia) {
        if constexpr (kDia) {
            if (t.rfn) { if (mask) GSIS_SWEEP(true, true, true); else GSIS_SWEEP(true, true, false); }
            else { if (mask) GSIS_SWEEP(true, false, true); else GSIS_SWEEP(true, false, false); }
        }
    } else {
        if (t.rfn) { if (mask) GSIS_SWEEP(false, true, true); else GSIS_SWEEP(false, true, false); }
        else { if (mask) GSIS_SWEEP(false, false, true); else GSIS_SWEEP(false, false, false); }
    }
#undef GSIS_SWEEP
}

template <typename T, int TX, int TY, int WX, int WY>
static void sweep_plane(const Target &t, int p, hipStream_t s)
{
    if (!t.nclean) {
        sweep_launch<T, TX, TY, WX, WY>(t, p, s, (unsigned)t.npblk[p], t.mask, -1);
        return;
    }
    // split: the clean entries without the solid-cell logic, then the rest
    const int nc = t.nclean[p], nd = 8 * t.pcnt[p] - nc;
    if (nc > 0) sweep_launch<T, TX, TY, WX, WY>(t, p, s, (unsigned)(nc * t.nvb), false, 0);
    if (nd > 0) sweep_launch<T, TX, TY, WX, WY>(t, p, s, (unsigned)(nd * t.nvb), true, nc);
}

bool sweep_shape_supported(bool fp32, bool dia, int tx, int ty)
{
    const Shape *sh = find_shape(fp32, tx, ty);
    if (!sh) return false;
    return !(dia && (tx / sh->wx) * (ty / sh->wy) > 32);
}

int sweep_shape_waves(bool fp32, int tx, int ty)
{
    const Shape *sh = find_shape(fp32, tx, ty);
    return sh ? sh->wx * sh->wy : 0;
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

hipError_t launch_sweep(const Target &t, hipStream_t s)
{
    const int tx = t.tx, ty = t.ty;
    if (!sweep_shape_supported(t.fp32, t.dia, tx, ty)) return hipErrorInvalidValue;
    const int nw = sweep_shape_waves(t.fp32, tx, ty);
    if (nw > 1 && t.bs != 64 * nw) return hipErrorInvalidValue;
    for (int p = 0; p < t.nplane; ++p) {
        if (t.npblk[p] == 0) continue;
        if (t.fp32) {
            if (tx == 4 && ty == 4) sweep_plane<float, 4, 4, 1, 1>(t, p, s);
            else if (tx == 8 && ty == 4) sweep_plane<float, 8, 4, 1, 1>(t, p, s);
            else if (tx == 8 && ty == 8) sweep_plane<float, 8, 8, 1, 1>(t, p, s);
            else sweep_plane<float, 8, 4, 2, 2>(t, p, s);
        } else {
            if (tx == 4 && ty == 4) sweep_plane<double, 4, 4, 1, 1>(t, p, s);
            else if (tx == 8 && ty == 4) sweep_plane<double, 8, 4, 1, 1>(t, p, s);
            else sweep_plane<double, 4, 4, 2, 2>(t, p, s);
        }
    }
    return hipGetLastError();
}

}  // namespace gsis

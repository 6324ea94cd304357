// Host-side launchers of the libgsis kernels (internal).
#pragma once
#include "gsis_common.h"

namespace gsis {

// Grid shapes of the kernels of a GSIS iteration; a launch over several cases
// concatenates the blocks each case needs (kind_blocks) through a block map.
enum Kind { K_CELL64, K_CELL128, K_CELL256, K_CELL1, K_FACE256, K_FACE8, K_GRAD, K_RES, K_CASE, NKIND };
int kind_blocks(const Geo &g, Kind k);

// What a launch covers: one case (maps null) or a batch of cases that share
// precision, gas and tile shape.
struct Target {
    const Case *cases = nullptr;      // device table
    int ncase = 1;
    const Case *host = nullptr;       // host copies of the table
    const int2 *map[NKIND] = {};      // device block maps (nullptr for one case)
    int nblk[NKIND] = {};             // grid size per kind
    const int2 *const *pmap = nullptr;   // sweep: block map of every global plane (nullptr for one case)
    const int *npblk = nullptr;          // sweep: blocks of every global plane
    int nplane = 0;
    // split sweep of one case with solid cells: per plane, the (tile, octant)
    // entries whose tile and upwind halo hold no solid cell (the first
    // nclean[p] of the plane's 8 pcnt[p] entries) run the kernel without the
    // solid-cell logic, the rest the masked one; nullptr: one kernel for all
    const int *nclean = nullptr, *pcnt = nullptr;
    int nvb = 0;
    bool fp32 = false, dia = false, mask = false, rfn = false;
    bool vlist = false;               // the node-list kernels (a refined or unstructured velocity mesh)
    bool g13 = false;                 // some case takes the Grad-13 wall flux in its correction
    // the moment kernel runs once per vector width (1, 2, 4) over the cases of that width
    const int2 *mom_map[3] = {};
    int mom_nblk[3] = {};
    int tx = 4, ty = 4, bs = 128;     // sweep tile shape and block size
    Span span(Kind k) const { return Span{cases, map[k]}; }
};

hipError_t launch_setup_tables(const Geo &g, const BcInfo &bc, const Dev &d, hipStream_t s);
hipError_t launch_init_maxwellian(const Geo &g, const Dev &d, bool fp32, double rho, const double *u, double Tt,
                                  double Tr, hipStream_t s);
hipError_t launch_to_canonical(const Geo &g, const Dev &d, bool fp32, const void *src, double *dst, hipStream_t s);
hipError_t launch_from_canonical(const Geo &g, const Dev &d, bool fp32, const double *src, void *dst, hipStream_t s);
hipError_t launch_vdf_node(const Geo &g, const Dev &d, bool fp32, int node, double *out, hipStream_t s);
hipError_t launch_apply_correction(const Geo &g, const Dev &d, bool fp32, hipStream_t s);
// order 2: limiter, then inv_dt f^n - (D2 - D1) into d.ho0/ho1, from the stored f^n
hipError_t launch_recon(const Geo &g, const Dev &d, bool fp32, hipStream_t s);

hipError_t launch_moments(const Target &t, hipStream_t s);
hipError_t launch_derive(const Target &t, hipStream_t s);
hipError_t launch_commit_correction(const Target &t, hipStream_t s);

hipError_t launch_params(const Target &t, hipStream_t s);
hipError_t launch_face_scale(const Target &t, hipStream_t s);

bool sweep_shape_supported(bool fp32, bool dia, int tx, int ty);
// waves of the wave grid serving tile (tx, ty): 1 for a single-wave slab, 0 if not compiled
int sweep_shape_waves(bool fp32, int tx, int ty);
int sweep_shapes(bool fp32, int *out, int max);
hipError_t launch_sweep(const Target &t, hipStream_t s);
// unstructured mesh: boundary-face density scales, then the sweep level by level
// (lev_off[L] .. lev_off[L + 1] are the entries of level L)
hipError_t launch_uface_scale(const Target &t, int pending, hipStream_t s);
hipError_t launch_usweep(const Target &t, const int *lev_off, int nlev, hipStream_t s);

// euler != 0: the Euler constitutive relations (no stress, heat flux, HoT or
// diffusive pseudo-time terms) and the iterate's own boundary flux
hipError_t launch_gsis_macro(const Target &t, int iters, hipStream_t s, int euler = 0);
// the same solve on an unstructured mesh (one case, centroids given)
hipError_t launch_umacro(const Target &t, int iters, hipStream_t s, int euler = 0);

int resid_blocks(const Geo &g);
hipError_t launch_zero_int(int *p, int n, hipStream_t s);
// red: partial-sum buffer [resid_blocks + 1][6]; nullptr = each case's workspace buffer
hipError_t launch_residual(const Target &t, hipStream_t s, double *red = nullptr);
// blocks of 256 cells the allocation-free residual can take, and the device
// address of its static partial-sum array on the current device
constexpr int RESID_STATIC_BLOCKS = 4096;
hipError_t resid_static_scratch(double **out);
hipError_t launch_snapshot(const Target &t, hipStream_t s);
hipError_t launch_hist_advance(int *ctr, hipStream_t s);

}  // namespace gsis

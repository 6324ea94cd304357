// Host-side launchers of the libgsis kernels (internal).
#pragma once
#include "gsis_common.h"

namespace gsis {

hipError_t launch_setup_tables(const Geo &g, const BcInfo &bc, const Dev &d, hipStream_t s);
hipError_t launch_init_maxwellian(const Geo &g, const Dev &d, bool fp32, double rho, const double *u, double Tt,
                                  double Tr, hipStream_t s);
hipError_t launch_to_canonical(const Geo &g, const Dev &d, bool fp32, const void *src, double *dst, hipStream_t s);
hipError_t launch_from_canonical(const Geo &g, const Dev &d, bool fp32, const double *src, void *dst, hipStream_t s);
hipError_t launch_vdf_node(const Geo &g, const Dev &d, bool fp32, int node, double *out, hipStream_t s);
hipError_t launch_apply_correction(const Geo &g, const Dev &d, bool fp32, hipStream_t s);

hipError_t launch_moments(const Geo &g, const Dev &d, bool fp32, int vw, hipStream_t s);
hipError_t launch_derive(const Geo &g, const Dev &d, hipStream_t s);
hipError_t launch_commit_correction(const Geo &g, const Dev &d, hipStream_t s);

hipError_t launch_params(const Geo &g, const Dev &d, hipStream_t s);
hipError_t launch_face_scale(const Geo &g, const BcInfo &bc, const Dev &d, hipStream_t s);

bool sweep_shape_supported(bool fp32, bool dia, int tx, int ty);
int sweep_shapes(bool fp32, int *out, int max);
hipError_t launch_sweep(const Geo &g, const Dev &d, bool fp32, int tx, int ty, int tz, int bs, const int *plane_off,
                        const int *plane_cnt, int nplane, hipStream_t s);

hipError_t launch_gsis_macro(const Geo &g, const BcInfo &bc, const Dev &d, int iters, hipStream_t s);

int resid_blocks(const Geo &g);
hipError_t launch_zero_int(int *p, int n, hipStream_t s);
hipError_t launch_residual(const Geo &g, const Dev &d, hipStream_t s);
hipError_t launch_snapshot(const Geo &g, const Dev &d, hipStream_t s);

}  // namespace gsis

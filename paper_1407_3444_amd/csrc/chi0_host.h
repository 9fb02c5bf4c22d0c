// chi0_host.h -- host-side checks and device-descriptor builders shared by the plan and the
// batch entry points.
#pragma once

#include "../../include/chi0.h"
#include "chi0_internal.h"

namespace chi0 {

// Validate a problem description and its base arrays (host-side, nothing enqueued).
chi0_status check_desc(const chi0_desc *d, const double *eps_k, const double *c_k);

// Device view of a validated description (band_hi <= 0 resolved to n_bands).
MeshDev make_mesh(const chi0_desc &d, const double *eps_k, const double *c_k);

// Validate one q against its description; *msg (static text) says what is wrong.
chi0_status check_q(const chi0_desc &d, const chi0_q &q, const char **msg);

// Device view of one q: mesh data plus wrapped shift, or the explicit k+q arrays.
QDev make_qdev(const MeshDev &M, const chi0_q &q, double *W);

// chi0_dynamic on a fixed device buffer of scratch_bytes (the no-allocation entry point): as many
// q-points per launch sequence as the buffer holds, no profile events, no allocation.
chi0_status dynamic_scratch(chi0_plan_t p, int32_t nq, const chi0_q *qs, int32_t nw, const double *omega,
                            void *scratch, size_t scratch_bytes, double *chi);

// Record a HIP runtime error on a plan; returns CHI0_E_DEVICE.
chi0_status plan_device_error(chi0_plan_t p, hipError_t e, const char *where);

}  // namespace chi0

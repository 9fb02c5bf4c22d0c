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

}  // namespace chi0

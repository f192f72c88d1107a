// Device side of the set-up phase, called from the host builder (plain pointers only).
#pragma once

#include <cstdint>

namespace amge {

// The shared data of the weighted local problems of the first agglomeration step (the
// host builder's KuhnPlan), flattened row-major; per-slot arrays hold 8 matrices one
// after the other.
struct KuhnPlanView {
    int nd;          // 1: H(curl) (RT and ND problems), 0: H(div) (RT only)
    int nI, nz;      // RT interior faces, RT null-space dimension
    int nIn, nzn;    // ND interior edges, ND null-space dimension
    const double *H, *h, *C;     // 8 x (nz x nz), 8 x (nz x 6), 8 x (6 x 6)
    const double *up, *Q2;       // nI x 6, nI x nz
    const double *CH, *G0, *Wn;  // 6 x 12, nI x 12, nIn x nI
    const double *Q2n;           // nIn x nzn
    const double *Mn, *Fn, *Cn;  // 8 x (nIn x nIn), 8 x (nIn x 12), 8 x (12 x 12)
};

// Weighted local problems of nagg agglomerates on the current device, one workgroup per
// agglomerate.  w: host, nagg x 16 (the ND weights of the eight hexes, then the RT
// weights).  Outputs, host arrays: U (nagg x nI x 6) RT interior values, elrt (nagg x
// 36) next-level RT element, and for nd: Un (nagg x nIn x 12), elnd (nagg x 144).
// Throws amge::Error (AMGE_ERR_NOT_SPD) if a reduced mass is not positive definite,
// AMGE_ERR_HIP / AMGE_ERR_OOM on runtime failures.
void kuhn_local_device(const KuhnPlanView& p, const double* w, int64_t nagg, double* U, double* elrt, double* Un,
                       double* elnd);

}  // namespace amge

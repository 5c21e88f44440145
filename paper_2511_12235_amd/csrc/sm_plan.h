// sm_plan.h -- the plan object behind the opaque sm_plan handle, shared by
// the API and solver translation units (host side only).
#pragma once

#include <mutex>
#include <vector>

#include "../../include/sm.h"
#include "sm_internal.h"

// Event-pair timing of individual dispatches (sm_timing_enable).
struct SmTiming {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> ev;  // pairs: 2 q, 2 q + 1
    std::vector<int> kernel;     // kernel id of pair q
    int used = 0;
    bool overflow = false;
};

struct sm_plan {
    int device;
    sm_precision prec;
    smk::DevGeom G;
    smk::LaunchCfg L;
    smk::RecLayout RL;  // workspace layout of the strip records (3D)
    double2 *d_trig;
    double *d_tau;
    int64_t n_vox, n_rays;
    SmTiming *tm;
    // strip records of every view chunk, kept on the device between calls
    // (sm_plan_keep_records); chunk c at rec_cache + c * RL.data_off
    void *rec_cache = nullptr;
};

namespace smk {
// Record an error message for sm_last_error() and return the status.
sm_status set_error(sm_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
// SM_OK when the plan's device is current.
sm_status check_plan_device(const sm_plan *p);

// Operator plumbing of sm_forward / sm_back (sm_api.hip), shared with the
// entry point that brings its own scratch memory.
// Bytes of the forward's volume buffer (prefix sums, max |x|) and of the
// adjoint's `groups` partial volumes, for `batch` volumes.
int64_t fwd_volume_bytes(const sm_plan *p, int64_t batch);
int64_t back_volume_bytes(const sm_plan *p, int64_t batch, int groups);
// Argument checks of an operator call other than its workspace (status and
// sm_last_error as the entry points).
sm_status check_operands(const sm_plan *p, const void *in, void *out, int32_t batch);
// 3D operators with the records of each chunk of RL.views views taken from
// the plan's kept copy or built into `recws` (RL.data_off bytes), and the
// volume buffer at `vol`.
hipError_t run_forward3d(const sm_plan *p, const RecLayout &RL, const void *x, void *y, int batch,
                         void *recws, void *vol, hipStream_t st);
hipError_t run_back3d(const sm_plan *p, const RecLayout &RL, const LaunchCfg &L, const void *y,
                      void *x, int batch, void *recws, void *vol, hipStream_t st);
hipError_t run_apply2d(const sm_plan *p, bool adjoint, const void *in, void *out, int batch,
                       hipStream_t st);
}  // namespace smk

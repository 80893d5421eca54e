// Stage timing by events that the kernels' own dispatches carry.
//
// A timed stage hands two events to the launches of the calling thread: the
// first launch takes `start` (the event then holds that kernel's begin
// time), every launch takes `stop` (so it ends up holding the end time of
// the stage's last kernel).  No marker packet goes between the kernels, so
// timing a stage does not stretch the step it measures.  Outside a timed
// stage both are null and launches go out plainly.  Not part of the C-ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace fetd_timing {

struct Pending {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};

// Per thread; defined in fetd_host.cpp.
Pending &pending();

}  // namespace fetd_timing

// hipLaunchKernelGGL, or hipExtLaunchKernelGGL with the pending events.
#define FETD_LAUNCH(kernel, grid, block, shmem, stream, ...)                                  \
    do {                                                                                      \
        ::fetd_timing::Pending &fetd_pending_ = ::fetd_timing::pending();                     \
        if (fetd_pending_.stop) {                                                             \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, fetd_pending_.start,    \
                                  fetd_pending_.stop, 0, __VA_ARGS__);                        \
            fetd_pending_.start = nullptr;                                                    \
        } else {                                                                              \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);              \
        }                                                                                     \
    } while (0)

// repro_batch_internal.hpp -- batch planning entry points shared inside
// librepro (the request loop plans its queries' aggregates as batch jobs
// without blocking the host).
#ifndef REPRO_BATCH_INTERNAL_HPP
#define REPRO_BATCH_INTERNAL_HPP

#include <stddef.h>

#include "repro.h"

namespace repro {
namespace batchx {

// Workspace bytes of a batch and bytes of its plan image (host).
bool plan_sizes(const repro_batch_job* jobs, int njobs, repro_key_t kt, repro_scalar_t vt, repro_scalar_t T,
                const repro_batch_config* cfg, size_t* workspace_bytes, size_t* image_bytes);

// Plans a batch into `image` (host memory, to be copied to the start of the
// workspace before the launch) and fills the plan.  No device work.
int plan_into(const repro_batch_job* jobs, int njobs, repro_key_t kt, repro_scalar_t vt, repro_scalar_t T,
              const repro_batch_config* cfg, void* image, size_t image_cap, void* workspace, size_t workspace_bytes,
              repro_batch_plan* plan);

// Enqueues the reset and persistent kernels of a planned batch.
int launch(const repro_batch_plan* plan, uint32_t* status, hipStream_t stream);

// Largest group count a job keeps in one workgroup's LDS at L levels.
int slice_limit(int L);

}  // namespace batchx
}  // namespace repro

#endif  // REPRO_BATCH_INTERNAL_HPP

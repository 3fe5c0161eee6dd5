// Optional HIP-event timing of the dominant kernels (enabled by pd_profile_enable).
#pragma once
#include <hip/hip_runtime.h>

namespace pd {

// Records a start event on `s` at construction and a stop event at destruction, when
// profiling is enabled; the pair is kept under kernel id `id` until pd_profile_read().
class ProfRange {
   public:
    ProfRange(int id, hipStream_t s);
    ~ProfRange();
    ProfRange(const ProfRange&) = delete;
    ProfRange& operator=(const ProfRange&) = delete;

   private:
    int id_;
    hipStream_t s_;
    hipEvent_t e0_ = nullptr;
    bool on_ = false;
};

}  // namespace pd

// sketch_apply kernels for FP32 input (instantiations of sk_apply_item.hpp).
#include "sk_apply_item.hpp"

namespace sk {

hipError_t launch_apply_f32(const Plan& plan, const ApplyArgs& a, hipStream_t st)
{
    return launch_vec<float>(plan, a, st);
}

hipError_t batched_f32(int bg, bool vec, bool dual, const BatchDesc* descs, int32_t count, int64_t total_items,
                      uint32_t* counter, int grid, int waves, size_t lds_bytes, hipStream_t st)
{
    return batched_typed<float>(bg, vec, dual, descs, count, total_items, counter, grid, waves, lds_bytes, st);
}

}  // namespace sk

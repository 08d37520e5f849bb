// lsb_batch_raw.hip -- persistent batched kernels of plans that hold raw-slice
// jobs (a cover split into slices [t0, t0 + n), as the frames of a clip).
// Same kernels as the header-only plans, with the raw-slice span compiled in.
#include "lsb_batch_device.hpp"

namespace lsb {

BatchFn batch_fn_raw(int unroll, int nt, int cls) { return batch_fn_for<true>(unroll, nt, cls); }

}  // namespace lsb

// fsr_batched.cpp -- host side of the batched path (persistent kernel).
#include "fsr_runtime.h"

namespace fsr {

void release_batch_state(BatchState& st) { st.reserved = nullptr; }

}  // namespace fsr

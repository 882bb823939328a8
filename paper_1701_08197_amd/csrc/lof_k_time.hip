// Dispatch of the SumThreshold-along-time kernels, one translation unit per
// (input kind, lane width) in lof_k_time_{i,f}{32,48,64}.hip.
#include "lof_kernel_table.hpp"

namespace lofk {
const void* kernel_time_int32();
const void* kernel_time_int48();
const void* kernel_time_int64();
const void* kernel_time_float32();
const void* kernel_time_float48();
const void* kernel_time_float64();
const void* kernel_time_float32_cx();
const void* kernel_time_pre_int(int lanes);
const void* kernel_time_pre_float(int lanes);

const void* kernel_time(bool integer, int lanes) {
  if (integer) return lanes == 32 ? kernel_time_int32() : (lanes == 48 ? kernel_time_int48() : kernel_time_int64());
  return lanes == 32 ? kernel_time_float32() : (lanes == 48 ? kernel_time_float48() : kernel_time_float64());
}

const void* kernel_time_cx() { return kernel_time_float32_cx(); }

const void* kernel_time_pre(bool integer, int lanes) {
  return integer ? kernel_time_pre_int(lanes) : kernel_time_pre_float(lanes);
}
}  // namespace lofk

// Pencil-pass kernels for one transform length, SSF_N, given on the compiler
// command line; the build compiles this file once per supported length.
#include "ssf_pass.hpp"

#ifndef SSF_N
#error "compile with -DSSF_N=<transform length>"
#endif

#define SSF_CAT2(a, b) a##b
#define SSF_CAT(a, b) SSF_CAT2(a, b)

// Instantiating the launcher in both compilation passes emits every pass
// kernel of this length into the device code object.
namespace ssf {
template hipError_t launch_any<SSF_N>(int, int, int, const PassArgs&, dim3, hipStream_t);
}  // namespace ssf

// The launcher table is host data.
#if !defined(__HIP_DEVICE_COMPILE__)
namespace ssf {
const KernelSet SSF_CAT(kernels_, SSF_N) = make_kernel_set<SSF_N>();
}  // namespace ssf
#endif

// Kernel launches that can carry start/stop events recorded by the
// dispatch itself: their interval is the kernel's execution alone, the
// duration a profiler's kernel trace reports (events recorded on the stream
// around a launch also take in the command processor's work between them).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <tuple>

namespace cvf {

// Null events: a plain launch.
struct DispatchEvents {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};

// Launch of kernel k on stream s; the arguments are converted to the
// kernel's parameter types.  Returns the launch status.
template <typename... A, typename... V>
hipError_t go(void (*k)(A...), dim3 grid, dim3 block, hipStream_t s, const DispatchEvents& ev, V... v)
{
    static_assert(sizeof...(A) == sizeof...(V), "kernel argument count");
    std::tuple<A...> args(v...);
    void* ptr[sizeof...(A)];
    std::apply([&ptr](auto&... x) {
        int i = 0;
        ((ptr[i++] = (void*)&x), ...);
    }, args);
    if (ev.start) return hipExtLaunchKernel((const void*)k, grid, block, ptr, 0, s, ev.start, ev.stop, 0);
    return hipLaunchKernel((const void*)k, grid, block, ptr, 0, s);
}

}  // namespace cvf

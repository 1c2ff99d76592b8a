// Kernel launch that records the kernel's own start/end into a HIP event pair
// (in the dispatch packet) when timing is requested, and is a plain launch
// otherwise (plain launches are also what HIP graph capture records).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#define MG_LAUNCH(K, G, B, S, E0, E1, ...)                                      \
    do {                                                                         \
        if (E0) hipExtLaunchKernelGGL(K, G, B, 0, S, E0, E1, 0, __VA_ARGS__);    \
        else hipLaunchKernelGGL(K, G, B, 0, S, __VA_ARGS__);                     \
    } while (0)

// Finishing the outer kernels' partial sums (internal interface).
//
// The three per-block partial arrays of an outer residual launch are summed in
// one fixed order whatever block runs the sum: that of a 1024-thread block (a
// strided sum per virtual thread, then a pairwise tree), so the separate
// finalize kernel and a kernel that finishes the sums in an extra block give
// the same bits.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace mg {

constexpr int kSumLanes = 1024;

struct SumsJob {
    const double* partials;  // arrays x count partial sums
    int count;               // 0: no job
    int arrays;
    double* out;             // out[slot + k], k < arrays
    int slot;
    double* host_out;        // pinned host mirror, or null
    double seq;              // nonzero: written to host_out[kHostFlagSlot] once the sums are visible
};

// Slot of the pinned host mirror that receives SumsJob::seq.
constexpr int kHostFlagSlot = 15;

// Every thread of the block calls it; sh holds kSumLanes doubles.
__device__ __forceinline__ void finish_sums(const SumsJob& job, double* sh) {
    const int nt = blockDim.x * blockDim.y * blockDim.z;
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    for (int k = 0; k < job.arrays; ++k) {
        const double* p = job.partials + (size_t)k * job.count;
        for (int v = tid; v < kSumLanes; v += nt) {
            double a = 0.0;
            for (int i = v; i < job.count; i += kSumLanes) a += p[i];
            sh[v] = a;
        }
        __syncthreads();
        for (int s = kSumLanes >> 1; s > 0; s >>= 1) {
            for (int v = tid; v < s; v += nt) sh[v] += sh[v + s];
            __syncthreads();
        }
        if (tid == 0) {
            job.out[job.slot + k] = sh[0];
            if (job.host_out) job.host_out[job.slot + k] = sh[0];
        }
        __syncthreads();
    }
    // The host may read the mirror without a stream event: make the sums
    // visible at system scope, then raise the flag the host polls.
    if (job.host_out && tid == 0) {
        __threadfence_system();
        if (job.seq != 0.0) {
            *reinterpret_cast<volatile double*>(job.host_out + kHostFlagSlot) = job.seq;
            __threadfence_system();
        }
    }
}

}  // namespace mg

// Point generation kernel: coordinates of a range of points as 0.32 fixed point
// (Sec. 3.1 of Shulman, "Quasi-Monte Carlo Radiative Transfer"), one lane per
// (point, dimension) pair, row-major [count][dims] output (coalesced writes).
#include <hip/hip_runtime.h>

#include "qrt_internal.h"

namespace qrt {

template <int KIND>
__global__ void __launch_bounds__(256) k_points(const SeqParams S, uint64_t first, uint64_t count, int dims,
                                                uint32_t *__restrict__ out)
{
    const uint64_t total = count * (uint64_t)dims;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t j = e / (uint64_t)dims;
        int d = (int)(e - j * (uint64_t)dims);
        out[e] = seq_point<KIND>(S, first + j, d);
    }
}

hipError_t launch_points(const SeqParams &S, int kind, uint64_t first, uint64_t count, int dims, uint32_t *out,
                         hipStream_t stream)
{
    uint64_t total = count * (uint64_t)dims;
    if (total == 0) return hipSuccess;
    uint64_t need = (total + 255) / 256;
    int blocks = (int)(need < 8192 ? need : 8192);
    switch (kind) {
    case SEQ_SOBOL: hipLaunchKernelGGL(k_points<SEQ_SOBOL>, dim3(blocks), dim3(256), 0, stream, S, first, count, dims, out); break;
    case SEQ_HALTON: hipLaunchKernelGGL(k_points<SEQ_HALTON>, dim3(blocks), dim3(256), 0, stream, S, first, count, dims, out); break;
    case SEQ_NIED2: hipLaunchKernelGGL(k_points<SEQ_NIED2>, dim3(blocks), dim3(256), 0, stream, S, first, count, dims, out); break;
    case SEQ_HAMMERSLEY: hipLaunchKernelGGL(k_points<SEQ_HAMMERSLEY>, dim3(blocks), dim3(256), 0, stream, S, first, count, dims, out); break;
    case SEQ_PHILOX: hipLaunchKernelGGL(k_points<SEQ_PHILOX>, dim3(blocks), dim3(256), 0, stream, S, first, count, dims, out); break;
    case SEQ_FAURE: hipLaunchKernelGGL(k_points<SEQ_FAURE>, dim3(blocks), dim3(256), 0, stream, S, first, count, dims, out); break;
    case SEQ_SOBOL_OWEN: hipLaunchKernelGGL(k_points<SEQ_SOBOL_OWEN>, dim3(blocks), dim3(256), 0, stream, S, first, count, dims, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace qrt

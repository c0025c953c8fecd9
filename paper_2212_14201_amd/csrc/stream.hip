// Streaming device copy: the measured bandwidth reference beside the HBM
// peak.  One 16-byte piece per thread with nontemporal loads and stores, the
// access shape that streams fastest on MI355X (the same one the plain gate
// kernels use), so that "fraction of the measured copy rate" compares like
// with like.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "internal.hpp"

namespace qvm {

typedef float sc_f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_stream_copy(const sc_f4* __restrict__ src, sc_f4* __restrict__ dst,
                                                     uint64_t pieces) {
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < pieces; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace qvm

using namespace qvm;

extern "C" qvm_status qvm_stream_copy(void* dst, const void* src, size_t bytes, void* stream) {
    if (!dst || !src) return fail(QVM_EARG, "stream copy: NULL pointer");
    if (bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16)
        return fail(QVM_EARG, "stream copy: bytes and pointers must be multiples of 16");
    const uint64_t pieces = bytes / 16;
    if (pieces == 0) return QVM_OK;
    const char* s = (const char*)src;
    const char* d = (const char*)dst;
    if (s < d + bytes && d < s + bytes) return fail(QVM_EARG, "stream copy: buffers overlap");
    // at most 2^23 blocks (a dispatch counts its threads in 32 bits); larger
    // copies loop
    const uint64_t blocks = std::min<uint64_t>((pieces + 255) / 256, 1ull << 23);
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (const sc_f4*)src, (sc_f4*)dst, pieces);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(QVM_EDEVICE, std::string("stream copy: ") + hipGetErrorString(e));
    return QVM_OK;
}

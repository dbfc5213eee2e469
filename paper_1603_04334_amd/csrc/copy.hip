// Reference copy kernel: the HBM bandwidth a plain streaming kernel reaches
// on this device, against which the step kernels' bandwidth is compared, and
// the known-size workload that calibrates the hardware traffic counters.
// Each lane moves one 16-byte unit with non-temporal loads and stores (the
// fastest plain copy measured on MI355X: 16-byte accesses reach about 1.7x
// the bandwidth of 4-byte ones).
#include "internal.hpp"

namespace sparc {

typedef unsigned CopyU4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) stream_copy_kernel(CopyU4 *__restrict__ dst, const CopyU4 *__restrict__ src,
                                                          long long n)
{
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace sparc

using namespace sparc;

extern "C" int sparc_stream_copy(void *dst, const void *src, size_t bytes, void *stream)
{
    if (!dst || !src) return fail(SPARC_E_ARG, "null pointer");
    if (bytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0)
        return fail(SPARC_E_ARG, "byte count and addresses must be multiples of 16");
    const char *s0 = (const char *)src, *d0 = (const char *)dst;
    if (s0 < d0 + bytes && d0 < s0 + bytes) return fail(SPARC_E_ALIAS, "source and destination overlap");
    const long long n = (long long)(bytes / 16);
    if (n == 0) return SPARC_OK;
    const long long blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffLL) return fail(SPARC_E_SHAPE, "copy too large for one launch");
    hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, (CopyU4 *)dst,
                       (const CopyU4 *)src, n);
    SPARC_HIP(hipGetLastError());
    return SPARC_OK;
}

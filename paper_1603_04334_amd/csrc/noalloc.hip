// H X without allocation: for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  The projector gather partials that sparc_h_apply keeps in a
// caller-supplied workspace live here in a fixed device array instead; the
// kernels are those of sparc_h_apply, so the results are bitwise the same.
#include <map>
#include <mutex>

#include "internal.hpp"

namespace sparc {
namespace {

constexpr size_t kScratchBytes = 16u << 20;  // 16 MiB per device

// A host-side stand-in only: device code addresses it, host code uses the
// per-device address returned by hipGetSymbolAddress.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;

// the scratch array's address on the current device, looked up once per device
int scratch_address(void **out)
{
    int dev = 0;
    SPARC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return SPARC_OK;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(SPARC_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
    *out = p;
    return SPARC_OK;
}

}  // namespace
}  // namespace sparc

using namespace sparc;

extern "C" size_t sparc_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int sparc_h_apply_noalloc(const sparc_op *op, int32_t dtype, const void *X, int64_t ldx, void *Y,
                                     int64_t ldy, int32_t ns, void *stream)
{
    if (!op) return fail(SPARC_E_ARG, "op is NULL");
    if (dtype != SPARC_F64 && dtype != SPARC_F32) return fail(SPARC_E_ARG, "dtype must be SPARC_F64 or SPARC_F32");
    if (ns < 1) return fail(SPARC_E_SHAPE, "ns must be >= 1");
    const size_t need = sparc_workspace_bytes(op, dtype, ns, 0);
    if (op->natoms > 0 && need > kScratchBytes)
        return fail(SPARC_E_WORKSPACE, "projections of " + std::to_string(ns) + " columns need " + std::to_string(need) +
                                           " bytes, more than the " + std::to_string(kScratchBytes) +
                                           "-byte scratch array");
    void *ws = nullptr;
    int st;
    if ((st = scratch_address(&ws))) return st;
    return sparc_h_apply(op, dtype, X, ldx, Y, ldy, ns, ws, kScratchBytes, stream);
}

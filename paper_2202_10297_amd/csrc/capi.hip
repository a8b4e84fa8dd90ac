// Library-level C-ABI entry points: error text, version, workspace clearing.
#include <string.h>

#include "common.h"
#include "prims.h"

namespace pvjp {

static thread_local char g_err[512];

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

__global__ void fill_zero_u32(uint32_t* __restrict__ p, int64_t nwords) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

}  // namespace pvjp

using namespace pvjp;

extern "C" const char* pvjp_last_error(void) { return g_err; }

extern "C" const char* pvjp_version(void) { return "pvjp 0.1.0 gfx950"; }

extern "C" pvjp_status pvjp_ws_clear(void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (ws_bytes == 0) return PVJP_OK;
    PVJP_REQUIRE(ws != nullptr, "pvjp_ws_clear: ws is NULL");
    PVJP_REQUIRE(aligned(ws, 4) && ws_bytes % 4 == 0, "pvjp_ws_clear: ws must be 4-byte aligned and sized");
    const int64_t nw = (int64_t)(ws_bytes / 4);
    hipLaunchKernelGGL(fill_zero_u32, dim3(flat_grid(nw, 256, 4)), dim3(256), 0, as_stream(stream),
                       (uint32_t*)ws, nw);
    PVJP_LAUNCHED("pvjp_ws_clear");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_ws_check(void* ws, int clear, void* stream) {
    clear_error();
    PVJP_REQUIRE(ws != nullptr && aligned(ws, 256), "pvjp_ws_check: ws must be non-NULL and 256-byte aligned");
    hipStream_t st = as_stream(stream);
    uint32_t err = 0;
    auto* hdr = reinterpret_cast<LookbackHdr*>(ws);
    if (hipMemcpyAsync(&err, &hdr->error, sizeof(err), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("pvjp_ws_check: reading the workspace header failed");
        return PVJP_EDEVICE;
    }
    if (err != 0) {
        if (clear) {
            const uint32_t zero = 0;
            if (hipMemcpyAsync(&hdr->error, &zero, sizeof(zero), hipMemcpyHostToDevice, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                set_error("pvjp_ws_check: clearing the workspace error failed");
                return PVJP_EDEVICE;
            }
        }
        set_error("pvjp_ws_check: lookback workspace error bits 0x%x (%s%s)", err,
                  (err & kErrTicket) ? "ticket outside the grid; " : "",
                  (err & kErrSpin) ? "a predecessor never published" : "");
        return PVJP_EDEVICE;
    }
    return PVJP_OK;
}

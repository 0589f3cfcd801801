// Allocation-free 2-D DCT-II / DCT-III (dctx_dct2d_noalloc): the plain 2-D
// transform of dctx_dct2d_ws with its workspace and its FP32 tables in one
// file-scope device array, so a call makes no hipMalloc / hipFree.
//
// Layout of `scratch` on every device (each device holds its own copy at its
// own address until the process ends):
//   [0, kWsBytes)                    workspace: the packed half spectrum (or
//                                    the transposed route's arrays), written
//                                    in full by each call before it is read;
//   [kWsBytes, kWsBytes + kTabBytes) table arena: the FP32 tables of the
//                                    shapes called so far (built in FP64 on
//                                    the host, copied in with hipMemcpy once
//                                    per shape, direction and norm).
// Host code never passes `scratch` itself to a kernel: on the host the name
// is a stand-in, not a device address.  Set-up (the first call on a device)
// asks the runtime for the device address with hipGetSymbolAddress and every
// launch uses that address.
#include <hip/hip_runtime.h>

#include <mutex>
#include <new>

#include "noalloc.h"

namespace {

constexpr size_t kWsBytes = DCTX_NOALLOC_WS_BYTES;   // 4096 x 4096: 4096 rows of 2048 complex values
constexpr size_t kTabBytes = (size_t)4 << 20;   // many times the tables of any one call
constexpr size_t kScratchBytes = kWsBytes + kTabBytes;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

// Per-device state: the device address of `scratch` and its table arena.
struct DeviceScratch {
    std::mutex mu;
    char *ptr = nullptr;   // device address of scratch on this device (set-up done when non-null)
    dctx::TableArena arena;
};
DeviceScratch g_dev[kMaxDevices];

dctx_status setup(DeviceScratch &d, int device) {
    if (d.ptr) return DCTX_OK;
    if (hipSetDevice(device) != hipSuccess) return DCTX_ERR_DEVICE;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return DCTX_ERR_DEVICE;
    d.ptr = static_cast<char *>(p);
    d.arena.base = d.ptr + kWsBytes;
    d.arena.cap = kTabBytes;
    d.arena.used = 0;
    return DCTX_OK;
}

}  // namespace

extern "C" {

dctx_status dctx_dct2d_noalloc(dctx_handle h, const float *x, float *y, int n1, int n2, dctx_norm norm,
                               int inverse, void *stream) {
    const int device = dctx::handle_device(h);
    if (device < 0 || !x || !y) return DCTX_ERR_INVALID;
    if (inverse != 0 && inverse != 1) return DCTX_ERR_INVALID;
    if (device >= kMaxDevices) return DCTX_ERR_UNSUPPORTED;
    if (n1 >= 1 && n2 >= 1 && dctx::ws_bytes_2d_plain_call(n1, n2) > kWsBytes) return DCTX_ERR_TOO_LARGE;
    try {
        DeviceScratch &d = g_dev[device];
        std::lock_guard<std::mutex> lock(d.mu);
        dctx_status st = setup(d, device);
        if (st != DCTX_OK) return st;
        st = dctx::run_2d_in_arena(h, x, y, n1, n2, norm, inverse != 0, d.ptr, kWsBytes, stream, &d.arena);
        if (st == dctx::kArenaFull) {
            // The arena is full: wait until no launch reads its tables, start
            // it over and run the call again (a transposed-route call may
            // already have enqueued its first transpose, which then runs twice
            // on the same stream with the same result).
            if (hipDeviceSynchronize() != hipSuccess) return DCTX_ERR_DEVICE;
            dctx::arena_clear(d.arena);
            st = dctx::run_2d_in_arena(h, x, y, n1, n2, norm, inverse != 0, d.ptr, kWsBytes, stream, &d.arena);
        }
        return st;
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

}  // extern "C"

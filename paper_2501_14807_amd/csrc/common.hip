// Status text, device check, fills and layer creation for libuvl.
#include <string.h>

#include <mutex>

#include "uvl_internal.h"

namespace uvl {
namespace {

// 16 bytes per thread, grid-stride; plain vector stores (graph-capture safe,
// unlike memset nodes).
__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t nv4 = n >> 2;
    uint4 *p4 = reinterpret_cast<uint4 *>(p);
    const uint4 val = make_uint4(v, v, v, v);
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nv4; k += stride) p4[k] = val;
    for (int64_t k = (nv4 << 2) + (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += stride) p[k] = v;
}

__global__ __launch_bounds__(kBlock) void k_zero_bytes(uint8_t *__restrict__ p, int64_t nbytes) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t n16 = nbytes >> 4;
    uint4 *p4 = reinterpret_cast<uint4 *>(p);
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n16; k += stride) p4[k] = make_uint4(0, 0, 0, 0);
    for (int64_t k = (n16 << 4) + (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nbytes; k += stride) p[k] = 0;
}

unsigned fill_grid(int64_t units) {
    int64_t g = ceil_div(units, kBlock);
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

void fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
    // p is 16-byte aligned by the callers' contracts
    hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid(n / 4 + 1)), dim3(kBlock), 0, s, p, n, v);
}

void fill_bytes(void *p, int64_t nbytes, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_bytes, dim3(fill_grid(nbytes / 16 + 1)), dim3(kBlock), 0, s,
                       static_cast<uint8_t *>(p), nbytes);
}

int32_t device_ok() {
    static std::mutex mu;
    static int32_t cached[64];
    static bool known[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return UVL_E_DEVICE;
    std::lock_guard<std::mutex> lock(mu);
    if (dev < 64 && known[dev]) return cached[dev];
    hipDeviceProp_t prop;
    int32_t st = UVL_E_DEVICE;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess)
        st = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? UVL_OK : UVL_E_UNSUPPORTED;
    if (dev < 64) {
        cached[dev] = st;
        known[dev] = true;
    }
    return st;
}

}  // namespace uvl

using namespace uvl;

extern "C" const char *uvl_status_str(int32_t status) {
    switch (status) {
        case UVL_OK: return "ok";
        case UVL_E_INVAL: return "invalid argument";
        case UVL_E_SHAPE: return "size mismatch";
        case UVL_E_DTYPE: return "bad dtype or label out of range";
        case UVL_E_NOMEM: return "workspace too small";
        case UVL_E_DEVICE: return "HIP error";
        case UVL_E_UNSUPPORTED: return "device is not gfx950";
        case UVL_E_RANGE: return "texel areas span too wide a range: build with area_w_hi";
        default: return "unknown status";
    }
}

extern "C" int32_t uvl_device_check(void) { return device_ok(); }

extern "C" int32_t uvl_create_layer(const uvl_layer *layer, void *stream) {
    if (!layer_ok(layer)) return UVL_E_INVAL;
    if (!dtype_ok(layer->dtype)) return UVL_E_DTYPE;
    if (int32_t s = device_ok()) return s;
    const int64_t n = (int64_t)layer->width * layer->height * (layer->dtype == UVL_U8 ? 1 : 2);
    fill_bytes(layer->data, n, as_stream(stream));
    return launch_status();
}

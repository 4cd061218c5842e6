// Layer pool for libuvl (§4.2: the Texture Manager sorts textures into
// texture arrays by a key joining width, height and data type, and sparse
// textures separate reserving address space from committing memory).
//
// On MI355X a layer is plain device memory, so the "texture array" of a key
// is one reserved virtual address range of `slots` layer-sized slots; slot k
// of key (w, h, dtype) lives at base + k * stride, stride being the layer's
// size rounded up to the device's allocation granularity.  Reserving costs
// no memory; creating a layer commits physical memory to a free slot
// (hipMemCreate, hipMemMap, hipMemSetAccess) and freeing it unmaps and
// releases it.  Kernels then address every layer of a key from one base
// pointer and a slot index, and a server can hold address space for many
// more layers than it has memory for.  This is the only part of the library
// that allocates device memory; everything else works on caller memory.
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "uvl_internal.h"

struct uvl_pool {
    struct Slab {
        char *base = nullptr;
        size_t stride = 0;
        std::vector<hipMemGenericAllocationHandle_t> handle;
        std::vector<bool> used;
    };
    int device = 0;
    int32_t slots = 0;
    size_t granularity = 0;
    uint64_t committed = 0;
    std::map<std::tuple<int32_t, int32_t, int32_t>, Slab> keys;
    mutable std::mutex mu;
};

namespace uvl {
namespace {

constexpr int32_t kMaxSlots = 65536;

hipMemAllocationProp device_prop(int device) {
    hipMemAllocationProp prop = {};
    prop.type = hipMemAllocationTypePinned;
    prop.location.type = hipMemLocationTypeDevice;
    prop.location.id = device;
    return prop;
}

bool key_ok(int32_t w, int32_t h, int32_t dt) {
    return w >= 1 && h >= 1 && w <= kMaxSide && h <= kMaxSide && dt >= UVL_U8 && dt <= UVL_F32;
}

// Unmap and release slot k of a slab (committed); false if HIP fails.  A
// slot whose unmap fails stays committed and in use (its mapping is still
// there); once unmapped, the slot is free again even if releasing the
// physical memory fails.
bool release_slot(uvl_pool *p, uvl_pool::Slab &s, int k) {
    if (hipMemUnmap(s.base + (size_t)k * s.stride, s.stride) != hipSuccess) return false;
    const bool rel = hipMemRelease(s.handle[k]) == hipSuccess;
    s.used[k] = false;
    p->committed -= s.stride;
    return rel;
}

}  // namespace
}  // namespace uvl

using namespace uvl;

extern "C" int32_t uvl_pool_create(int32_t slots_per_key, uvl_pool **out) {
    if (!out || slots_per_key < 1 || slots_per_key > kMaxSlots) return UVL_E_INVAL;
    *out = nullptr;
    if (int32_t s = device_ok()) return s;
    int dev = 0, vmm = 0;
    if (hipGetDevice(&dev) != hipSuccess) return UVL_E_DEVICE;
    if (hipDeviceGetAttribute(&vmm, hipDeviceAttributeVirtualMemoryManagementSupported, dev) != hipSuccess)
        return UVL_E_DEVICE;
    if (!vmm) return UVL_E_UNSUPPORTED;
    const hipMemAllocationProp prop = device_prop(dev);
    size_t gran = 0;
    if (hipMemGetAllocationGranularity(&gran, &prop, hipMemAllocationGranularityMinimum) != hipSuccess || gran == 0)
        return UVL_E_DEVICE;
    uvl_pool *p = new uvl_pool;
    p->device = dev;
    p->slots = slots_per_key;
    p->granularity = gran;
    *out = p;
    return UVL_OK;
}

extern "C" int32_t uvl_pool_alloc(uvl_pool *p, int32_t width, int32_t height, int32_t dtype, void **data,
                                  int32_t *slot) {
    if (!p || !data) return UVL_E_INVAL;
    if (width < 1 || height < 1 || width > kMaxSide || height > kMaxSide) return UVL_E_INVAL;
    if (!key_ok(width, height, dtype)) return UVL_E_DTYPE;
    std::lock_guard<std::mutex> lock(p->mu);
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || cur != p->device) return UVL_E_DEVICE;
    auto key = std::make_tuple(width, height, dtype);
    auto it = p->keys.find(key);
    if (it == p->keys.end()) {
        uvl_pool::Slab s;
        const size_t bytes = (size_t)width * height * dtype_bytes(dtype);
        s.stride = (size_t)ceil_div((int64_t)bytes, (int64_t)p->granularity) * p->granularity;
        void *base = nullptr;
        if (hipMemAddressReserve(&base, s.stride * (size_t)p->slots, 0, nullptr, 0) != hipSuccess) return UVL_E_NOMEM;
        s.base = static_cast<char *>(base);
        s.handle.assign(p->slots, hipMemGenericAllocationHandle_t{});
        s.used.assign(p->slots, false);
        it = p->keys.emplace(key, std::move(s)).first;
    }
    uvl_pool::Slab &s = it->second;
    int k = 0;
    while (k < p->slots && s.used[k]) ++k;
    if (k == p->slots) return UVL_E_NOMEM;
    const hipMemAllocationProp prop = device_prop(p->device);
    hipMemGenericAllocationHandle_t h{};
    const hipError_t e = hipMemCreate(&h, s.stride, &prop, 0);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? UVL_E_NOMEM : UVL_E_DEVICE;
    char *ptr = s.base + (size_t)k * s.stride;
    if (hipMemMap(ptr, s.stride, 0, h, 0) != hipSuccess) {
        (void)hipMemRelease(h);      // already failing: the first error is reported
        return UVL_E_DEVICE;
    }
    hipMemAccessDesc access = {};
    access.location.type = hipMemLocationTypeDevice;
    access.location.id = p->device;
    access.flags = hipMemAccessFlagsProtReadWrite;
    if (hipMemSetAccess(ptr, s.stride, &access, 1) != hipSuccess) {
        (void)hipMemUnmap(ptr, s.stride);
        (void)hipMemRelease(h);
        return UVL_E_DEVICE;
    }
    s.handle[k] = h;
    s.used[k] = true;
    p->committed += s.stride;
    *data = ptr;
    if (slot) *slot = k;
    return UVL_OK;
}

extern "C" int32_t uvl_pool_free(uvl_pool *p, void *data) {
    if (!p || !data) return UVL_E_INVAL;
    std::lock_guard<std::mutex> lock(p->mu);
    char *c = static_cast<char *>(data);
    for (auto &kv : p->keys) {
        uvl_pool::Slab &s = kv.second;
        if (c < s.base || c >= s.base + s.stride * (size_t)p->slots) continue;
        const size_t off = (size_t)(c - s.base);
        const int k = (int)(off / s.stride);
        if (off % s.stride || !s.used[k]) return UVL_E_INVAL;
        // Unmapping is not ordered against queued kernels: wait for every
        // stream of the pool's device before the memory goes away.
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess || cur != p->device) return UVL_E_DEVICE;
        if (hipDeviceSynchronize() != hipSuccess) return UVL_E_DEVICE;
        return release_slot(p, s, k) ? UVL_OK : UVL_E_DEVICE;
    }
    return UVL_E_INVAL;
}

extern "C" int32_t uvl_pool_array(const uvl_pool *p, int32_t width, int32_t height, int32_t dtype, void **base,
                                  size_t *stride, int32_t *slots) {
    if (!p || !base || !stride || !slots) return UVL_E_INVAL;
    std::lock_guard<std::mutex> lock(p->mu);
    auto it = p->keys.find(std::make_tuple(width, height, dtype));
    if (it == p->keys.end()) return UVL_E_INVAL;
    *base = it->second.base;
    *stride = it->second.stride;
    *slots = p->slots;
    return UVL_OK;
}

extern "C" int32_t uvl_pool_stats(const uvl_pool *p, uint64_t *reserved, uint64_t *committed, int32_t *keys) {
    if (!p || !reserved || !committed || !keys) return UVL_E_INVAL;
    std::lock_guard<std::mutex> lock(p->mu);
    uint64_t r = 0;
    for (const auto &kv : p->keys) r += kv.second.stride * (uint64_t)p->slots;
    *reserved = r;
    *committed = p->committed;
    *keys = (int32_t)p->keys.size();
    return UVL_OK;
}

extern "C" int32_t uvl_pool_destroy(uvl_pool *p) {
    if (!p) return UVL_E_INVAL;
    bool ok = true;
    {
        std::lock_guard<std::mutex> lock(p->mu);
        int cur = 0;
        ok = hipGetDevice(&cur) == hipSuccess && cur == p->device && hipDeviceSynchronize() == hipSuccess;
        for (auto &kv : p->keys) {
            uvl_pool::Slab &s = kv.second;
            for (int k = 0; k < p->slots; ++k)
                if (s.used[k]) ok = release_slot(p, s, k) && ok;
            ok = hipMemAddressFree(s.base, s.stride * (size_t)p->slots) == hipSuccess && ok;
        }
    }
    delete p;
    return ok ? UVL_OK : UVL_E_DEVICE;
}

// Where an edit's selection goes (libuvl internal).
//
// The edit kernels (brush, lasso, screen-space tool) compute which texels a
// tool selects and hand each group of 4 consecutive texels to a sink:
//  - LabelSink stores a label in a label layer (§4.2 database layers hold
//    unsigned keys; 0 is the null key);
//  - ValueSink writes a numeric layer (§4.2 numeric layers pair the data
//    texture with a mask texture of validity flags): SET stores the value's
//    bit pattern and sets the texels' mask bits, ERASE clears the mask bits
//    and leaves the data.  The mask holds texel t in bit t % 32 of word
//    t / 32, so one word covers 32 consecutive texels.
// A kernel calls put4 with every lane of the wave active and 4-aligned t
// inside the atlas, put_some / put1 from divergent tail code.  `group_word`
// (wave-uniform) says that lanes 8g .. 8g+7 of the wave hold the 32 texels
// of one mask word in lane order, so that they merge their bits and one lane
// updates the word.
#pragma once

#include "uvl_internal.h"

namespace uvl {

// Store v in the selected texels of t .. t+3 (t 4-aligned, T-array 16-byte
// aligned); a full group is one vector store.
template <typename T>
__device__ __forceinline__ void store4(T *__restrict__ L, int64_t t, const bool s[4], T v) {
    if (s[0] && s[1] && s[2] && s[3]) {
        if constexpr (sizeof(T) == 1) {
            *reinterpret_cast<uint32_t *>(L + t) = 0x01010101u * v;
        } else if constexpr (sizeof(T) == 2) {
            const uint32_t w = 0x00010001u * v;
            *reinterpret_cast<uint2 *>(L + t) = make_uint2(w, w);
        } else {
            *reinterpret_cast<uint4 *>(L + t) = make_uint4(v, v, v, v);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (s[k]) L[t + k] = v;
    }
}

template <typename T>
struct LabelSink {
    T *L;
    T label;

    __device__ __forceinline__ void put4(int64_t t, const bool s[4], bool) const { store4<T>(L, t, s, label); }
    __device__ __forceinline__ void put_some(int64_t t, int nvalid, const bool s[4]) const {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nvalid && s[k]) L[t + k] = label;
    }
    __device__ __forceinline__ void put1(int64_t t) const { L[t] = label; }
};

// T is the storage width (uint8_t, uint16_t or uint32_t); `bits` is the
// value already converted to the layer's dtype on the host.
template <typename T>
struct ValueSink {
    T *D;
    uint32_t *mask;
    T bits;
    int32_t erase;

    __device__ __forceinline__ void word(uint32_t *p, uint32_t w) const {
        if (erase)
            atomicAnd(p, ~w);
        else
            atomicOr(p, w);
    }
    __device__ __forceinline__ void put4(int64_t t, const bool s[4], bool group_word) const {
        if (!erase) store4<T>(D, t, s, bits);
        const uint32_t nib = (uint32_t)s[0] | (uint32_t)s[1] << 1 | (uint32_t)s[2] << 2 | (uint32_t)s[3] << 3;
        if (group_word) {
            uint32_t w = nib << (t & 31);
            w |= __shfl_xor(w, 1, 8);
            w |= __shfl_xor(w, 2, 8);
            w |= __shfl_xor(w, 4, 8);
            if ((t & 31) == 0 && w) word(mask + (t >> 5), w);
        } else if (nib) {
            word(mask + (t >> 5), nib << (t & 31));   // t 4-aligned: the 4 bits share a word
        }
    }
    __device__ __forceinline__ void put1(int64_t t) const {
        if (!erase) D[t] = bits;
        word(mask + (t >> 5), 1u << (t & 31));
    }
    __device__ __forceinline__ void put_some(int64_t t, int nvalid, const bool s[4]) const {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nvalid && s[k]) put1(t + k);
    }
};

// Host side: call f with the sink of a label layer (u8 or u16, label
// already checked to fit) or of a numeric layer (bits from encode_value).
template <typename F>
void with_label_sink(const uvl_layer *l, uint32_t label, F &&f) {
    if (l->dtype == UVL_U8)
        f(LabelSink<uint8_t>{static_cast<uint8_t *>(l->data), (uint8_t)label});
    else
        f(LabelSink<uint16_t>{static_cast<uint16_t *>(l->data), (uint16_t)label});
}

template <typename F>
void with_value_sink(const uvl_numeric *l, uint32_t bits, int32_t mode, F &&f) {
    const int32_t erase = mode == UVL_ERASE;
    switch (dtype_bytes(l->dtype)) {
    case 1: f(ValueSink<uint8_t>{static_cast<uint8_t *>(l->data), l->mask, (uint8_t)bits, erase}); break;
    case 2: f(ValueSink<uint16_t>{static_cast<uint16_t *>(l->data), l->mask, (uint16_t)bits, erase}); break;
    default: f(ValueSink<uint32_t>{static_cast<uint32_t *>(l->data), l->mask, bits, erase}); break;
    }
}

}  // namespace uvl

// Device-memory access shared by the 2D and 3D kernels of liblb: global
// address-space pointers, buffer resources over row blocks, typed buffer
// loads and stores, and the storage traits (element type in memory,
// arithmetic type, encoding) of the four storage modes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lb_internal.hpp"

// Tuning switches (compile-time).
#ifndef LBK_ALT_DIR
#define LBK_ALT_DIR 1
#endif
#ifndef LBK_HALO_SPLIT
#define LBK_HALO_SPLIT 1
#endif
#ifndef LBK_PIPE
#define LBK_PIPE 1
#endif
#ifndef LBK_NT_STORE
#define LBK_NT_STORE 1
#endif

namespace lbk {

// ---------------------------------------------------------------------------
// Pointers into device global memory (address space 1).  The population
// buffers are reached through the member table, so without this the compiler
// cannot tell them from LDS and falls back to flat accesses.
#define LBK_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ LBK_GLOBAL T *gp(void *p) { return (LBK_GLOBAL T *)p; }

// Element at a uniform base plus a per-lane 32-bit byte offset: the form the
// hardware addresses with a scalar base register and one vector register.
template <class T>
__device__ __forceinline__ T ldg(const LBK_GLOBAL T *base, unsigned byte_off)
{
    return *(const LBK_GLOBAL T *)((const LBK_GLOBAL char *)base + byte_off);
}
template <class T>
__device__ __forceinline__ LBK_GLOBAL T *at(LBK_GLOBAL T *base, unsigned byte_off)
{
    return (LBK_GLOBAL T *)((LBK_GLOBAL char *)base + byte_off);
}

// Buffer resources.  Populations are stored in row blocks: the 18 segments
// f_i^s(., y) of lattice row y are adjacent, so one 128-bit resource spans a
// whole row block; a load adds a uniform byte offset (which population) and a
// per-lane byte offset (which column).  Accesses outside the resource read 0
// and write nothing.
constexpr int BUF_RAW_DWORD3 = 0x00020000;   // raw (untyped) buffer, gfx9 descriptor word 3
constexpr int CPOL_NT = 2;                   // non-temporal cache policy bit

using rsrc_t = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ rsrc_t row_rsrc(const void *buf, int row, int64_t row_bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)((const char *)buf + (int64_t)row * row_bytes), 0,
                                             (int)row_bytes, BUF_RAW_DWORD3);
}

template <class T> __device__ __forceinline__ T bload(rsrc_t r, unsigned voff, unsigned soff);
template <> __device__ __forceinline__ double bload<double>(rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <> __device__ __forceinline__ float bload<float>(rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <> __device__ __forceinline__ _Float16 bload<_Float16>(rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
}
template <> __device__ __forceinline__ uint16_t bload<uint16_t>(rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
}

template <int AUX>
__device__ __forceinline__ void bstore(double v, rsrc_t r, unsigned voff, unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                          voff, soff, AUX);
}
template <int AUX>
__device__ __forceinline__ void bstore(float v, rsrc_t r, unsigned voff, unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, AUX);
}
template <int AUX>
__device__ __forceinline__ void bstore(_Float16 v, rsrc_t r, unsigned voff, unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, voff, soff, AUX);
}
template <int AUX>
__device__ __forceinline__ void bstore(uint16_t v, rsrc_t r, unsigned voff, unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b16(v, r, voff, soff, AUX);
}

// ---------------------------------------------------------------------------
// Storage traits: element type T in memory, arithmetic type C of the
// collision, and SITE: whether the codes are shifted by each site's own
// density (the 16-bit modes, see below).
template <int ST> struct Tr;

template <> struct Tr<ST_F64> {
    using T = double;
    using C = double;
    static constexpr bool SITE = false;
    static __device__ __forceinline__ C dec(T v) { return v; }
    static __device__ __forceinline__ T enc(C v) { return v; }
};

template <> struct Tr<ST_F32> {
    using T = float;
    using C = float;
    static constexpr bool SITE = false;
    static __device__ __forceinline__ C dec(T v) { return v; }
    static __device__ __forceinline__ T enc(C v) { return v; }
};

// The 16-bit modes store, per site x and component s, the FP32 density
// rhat_s(x) and for every population a code q_i = (f*_i - w_i r) S_i rounded
// to the 16-bit format (r: the site density rounded to FP32, S_i a power of
// two); a population decodes as f*_i = w_i rhat + q_i / S_i.  rhat is chosen
// so that the decoded populations of a site sum to its density (see
// site_encode in lb_kernels.hpp).  code() rounds a scaled residual to the
// format, value() returns the code as FP32 (exact).

// IEEE binary16 codes.
template <> struct Tr<ST_F16S> {
    using T = _Float16;
    using C = float;
    static constexpr bool SITE = true;
    static __device__ __forceinline__ T code(float x) { return (_Float16)x; }
    static __device__ __forceinline__ float value(T v) { return (float)v; }
};

// bfloat16 codes (kept as raw 16-bit patterns); the conversion rounds to
// nearest even (gfx950 converts in hardware).
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

template <> struct Tr<ST_BF16S> {
    using T = uint16_t;
    using C = float;
    static constexpr bool SITE = true;
    static __device__ __forceinline__ T code(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
    static __device__ __forceinline__ float value(T v) { return bf16_to_f32(v); }
};

}  // namespace lbk

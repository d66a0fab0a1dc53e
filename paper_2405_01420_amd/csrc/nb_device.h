// Device helpers shared by the force, adjoint and pair-export kernels, so that every kernel
// forms displacements and squared distances with bit-identical FP32 arithmetic.
#pragma once

#include "nb_internal.h"

// Periodic shift t in {-1, 0, 1}^3 from its index 9 (tx+1) + 3 (ty+1) + (tz+1).
__device__ __forceinline__ int nb_tx(int s) { return s / 9 - 1; }
__device__ __forceinline__ int nb_ty(int s) { return (s / 3) % 3 - 1; }
__device__ __forceinline__ int nb_tz(int s) { return s % 3 - 1; }

// Offsets that place the pair (i, j + t L) in one frame without rounding: the coordinate that
// lies near the upper box face is the one moved down by L, so both x - L steps are exact
// (Sterbenz) and d = (x_i + di) - (x_j + dj) carries a single rounding.
//   t = +1: j image near 0 seen from i near L  -> di = -L, dj = 0
//   t = -1: j near L seen from i near 0        -> di = 0,  dj = -L
// (Integer selects of the bit patterns: with a wave-uniform t they stay on the scalar unit.)
__device__ __forceinline__ float nb_di(int t, float L) {
    return __uint_as_float(t > 0 ? __float_as_uint(L) ^ 0x80000000u : 0u);
}
__device__ __forceinline__ float nb_dj(int t, float L) {
    return __uint_as_float(t < 0 ? __float_as_uint(L) ^ 0x80000000u : 0u);
}

__device__ __forceinline__ float nb_r2(float dx, float dy, float dz) {
    return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

// Hardware reciprocal square root and reciprocal (about 1 ulp) followed by one Newton step, so
// that the result carries only the rounding of the last fused multiply-add.  A systematic bias
// of the raw instruction would otherwise be amplified twelve-fold in r^-12 energy sums.
__device__ __forceinline__ float nb_rsq(float x) {
    const float y = __builtin_amdgcn_rsqf(x);
    const float h = x * y;
    const float e = __builtin_fmaf(-h, y, 1.0f);   // 1 - x y^2
    return __builtin_fmaf(0.5f * y, e, y);
}

__device__ __forceinline__ float nb_rcp(float x) {
    const float y = __builtin_amdgcn_rcpf(x);
    const float e = __builtin_fmaf(-x, y, 1.0f);
    return __builtin_fmaf(y, e, y);
}

// Global-memory (address space 1) pointers.  Pointers that the force body receives from a
// descriptor in memory would otherwise be generic, and every access through them a flat
// instruction; typed as global, the accesses compile to global loads, stores and atomics.
#define NB_G __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const NB_G T *nb_g(const T *p) { return (const NB_G T *)p; }
template <class T>
__device__ __forceinline__ NB_G T *nb_g(T *p) { return (NB_G T *)p; }
template <class T>
__device__ __forceinline__ T nb_ld(const NB_G T *p) { return *(const T *)p; }
template <class T>
__device__ __forceinline__ void nb_st(NB_G T *p, const T &v) { *(T *)p = v; }

// LDS (address space 3) accesses by byte address, for work areas addressed from packed codes.
#define NB_L __attribute__((address_space(3)))
__device__ __forceinline__ uint32_t nb_laddr(const void *p) {
    return (uint32_t)(size_t)(const NB_L void *)p;
}
// (The generic pointer made from the LDS one is turned back into LDS accesses by the compiler;
// HIP's vector types have no operators on address-space-qualified references.)
template <class T>
__device__ __forceinline__ T nb_lget(uint32_t a) { return *(const T *)(const NB_L T *)(size_t)a; }
template <class T>
__device__ __forceinline__ void nb_lput(uint32_t a, const T &v) { *(T *)(NB_L T *)(size_t)a = v; }

// Wave-local ordering of LDS writes before reads by other lanes of the same wavefront (the
// hardware executes one wave's LDS instructions in order; this keeps the compiler from moving
// them across).
__device__ __forceinline__ void nb_wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A value in a vector register that the compiler treats as unknown: bit masks used as VOP3
// operands (which take no literal constant) stay in registers instead of splitting the op.
__device__ __forceinline__ uint32_t nb_vreg(uint32_t v) {
    uint32_t r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(v));
    return r;
}

// The C mask bits of j-atom b of an entry (bit k: i-atom k interacts with j-atom b).
template <int C>
__device__ __forceinline__ unsigned nb_mask_column(uint32_t m, int b) {
    return (m >> (b * C)) & ((1u << C) - 1u);
}

// DPP move of x within 16-lane rows (CTRL: the DPP control word; rows not in ROW_MASK read 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float nb_dpp(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, false));
}

// Reduce-scatter of per-lane partial sums over the 64 lanes.  nb_fold32(a, b): a summed over the
// lane pairs (l, l + 32) into lanes 0-31 and b into lanes 32-63 (one v_permlane32_swap moves the
// upper half of a and the lower half of b across); nb_fold16 the same over (l, l ^ 16) within each
// half, a into the rows with bit 4 clear; nb_fold8 over (l, l ^ 8) within each 16-lane row.
__device__ __forceinline__ float nb_fold32(float a, float b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float nb_fold16(float a, float b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float nb_fold8(float a, float b, int lane) {
    const bool hi = (lane & 8) != 0;
    const float u = hi ? b : a, w = hi ? a : b;
    return u + nb_dpp<0x128, 0xf>(w);  // row_ror:8
}

// The C per-lane values v[k] summed over the 64 lanes: value k ends up in every lane of the
// group of 64 / C lanes with lane / (64 / C) == k.
template <int C>
__device__ __forceinline__ float nb_wave_scatter_sum(const float (&v)[C], int lane) {
    static_assert(C == 4 || C == 8, "clusters of 4 or 8 atoms");
    float t;
    if constexpr (C == 8) {
        const float a0 = nb_fold32(v[0], v[4]), a1 = nb_fold32(v[1], v[5]);
        const float a2 = nb_fold32(v[2], v[6]), a3 = nb_fold32(v[3], v[7]);
        t = nb_fold8(nb_fold16(a0, a2), nb_fold16(a1, a3), lane);
    } else {
        t = nb_fold16(nb_fold32(v[0], v[2]), nb_fold32(v[1], v[3]));
        t += nb_dpp<0x128, 0xf>(t);  // row_ror:8
    }
    t += nb_dpp<0xB1, 0xf>(t);   // quad_perm [1,0,3,2]
    t += nb_dpp<0x4E, 0xf>(t);   // quad_perm [2,3,0,1]
    t += nb_dpp<0x141, 0xf>(t);  // row_half_mirror
    return t;
}


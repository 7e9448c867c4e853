// k_common.h -- device helpers shared by the libgpr kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace gpr {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Loads and stores through pointers that address device memory. Pointers read
// from task descriptors have no known address space, so plain accesses
// compile to flat instructions; a flat load also counts against the LDS
// counter, and the wait for an LDS read then waits for it too (a prefetch
// from HBM would stall the MFMA loop). These go through the global address
// space instead.
template <typename T>
__device__ inline T gld(const T* p)
{
    return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ inline void gst(T* p, T v)
{
    *(__attribute__((address_space(1))) T*)p = v;
}
// Two consecutive doubles (16-byte aligned) as one global load; HIP's
// double2 is a class whose copy would go through a generic reference.
typedef double dbl2v __attribute__((ext_vector_type(2)));
__device__ inline double2 gld2(const double* p)
{
    const dbl2v v = *(const __attribute__((address_space(1))) dbl2v*)p;
    return make_double2(v.x, v.y);
}

// MI355X has 8 XCDs, each with its own L2; consecutive workgroup ids are
// dealt round-robin to the XCDs. This maps the hardware id to a logical id so
// that logical ids [x*q, (x+1)*q) all run on XCD x: the workgroups of one
// tile task (which share their A and B operands) then share one L2.
__device__ inline int xcd_remap(int b, int n)
{
    constexpr int NX = 8;
    const int q = n / NX, r = n % NX;
    const int x = b % NX, i = b / NX;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// D = A * B + C on 16 x 16 x 4 FP64 MFMA. Lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; element v of lane l is D[4 v + l / 16][l % 16]
// (rows interleaved across the four lane groups; measured on gfx950).
__device__ inline dbl4 mfma16(double a, double b, dbl4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row of element v held by a lane of group lk = l / 16 in an FP64 16 x 16 result.
__device__ constexpr int drow(int lk, int v) { return 4 * v + lk; }

// Value of x held by lane `l` (uniform result).
__device__ inline double lane_bcast(double x, int l)
{
    int lo = __double2loint(x), hi = __double2hiint(x);
    lo = __builtin_amdgcn_readlane(lo, l);
    hi = __builtin_amdgcn_readlane(hi, l);
    return __hiloint2double(hi, lo);
}

// Orders the LDS accesses of one wavefront around this point (no workgroup
// barrier): the empty asm with a memory clobber stops the compiler from
// moving memory accesses across it, and the LDS executes one wave's accesses
// in issue order, so a lane's read after it sees another lane's earlier write.
__device__ inline void wave_lds_sync()
{
    __asm__ __volatile__("" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

}  // namespace gpr

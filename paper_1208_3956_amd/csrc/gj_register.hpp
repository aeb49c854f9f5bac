// Gauss-Jordan inversion of a 64 x 64 complex block held in registers (FP64), shared by
// the strip factorisation (2-D) and the complex64 slab factorisation (3-D), where it
// inverts the diagonal blocks.
#pragma once
#include "helm_internal.hpp"

namespace helm {
namespace gjr {

// ---------------------------------------------------------------- register Gauss-Jordan
// Layout: lane i holds row i; wave g holds columns j = g + 4 r, r = 0..15, in M[r].  A step k
// pivots on column k (wave k % 4) at the unused row p of largest modulus and eliminates
// column k from every other row.  No rows are swapped and the pivot row is not scaled at
// its step: row p keeps its values (its column-k entry becomes 1) and is multiplied by its
// reciprocal pivot after the last step, which leaves every elimination unchanged because the
// updates are linear in the pivot row.  The finished array holds the inverse with row i at
// position step(i) (the step that pivoted on row i) and column j at position perm(j) (the row
// pivoted at step j).  The columns cycle through the registers: after every four steps the
// array is rotated by one register, so the column of the current step is always M[0].
struct GJShared {
    double2 fcol[2][WP];     // pivot column of the step (double-buffered: one barrier per step)
    int piv[2];
    int perm[WP];
};

// wavefront maximum (device library; declared by the HIP headers only on request)
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_max_u64(unsigned long long);

// component-wise select (a select of whole double2 values goes through scratch memory)
__device__ inline double2 sel(bool c, double2 a, double2 b) {
    return cmk<double2>(c ? a.x : b.x, c ? a.y : b.y);
}

__device__ inline double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Inverse of the leading W x W block of the matrix in M (zero elsewhere), written column-major
// with leading dimension WP to dst (zero outside the leading block); ends with a barrier so
// that dst can be read back by the workgroup.  Sets err when a pivot is zero or not finite.
__device__ inline void gj_invert_store(double2 (&M)[16], int W, GJShared& sh, double2* __restrict__ dst,
                                float2* __restrict__ dst32, int* err) {
    const int i = threadIdx.x & (WP - 1), g = threadIdx.x >> 6;
    bool used = i >= W;
    int my_step = i;                               // rows beyond W keep their position
    double2 my_inv = cmk<double2>(1.0, 0.0);
    int rot = 0;                                   // rotations done: M[r] holds column g + 4 (r + rot)
    for (int kk = 0; 4 * kk < W; ++kk) {
#pragma unroll
        for (int gg = 0; gg < 4; ++gg) {
            const int k = 4 * kk + gg;
            if (k < W) {
                const int buf = k & 1;
                if (g == gg) {
                    // pivot search over the unused rows: the key orders by |m|^2 (its low 6
                    // mantissa bits replaced by 63 - row, so ties go to the lower row)
                    const double2 v = M[0];
                    const double mag = v.x * v.x + v.y * v.y;
                    const unsigned long long key =
                        used ? 0ull : (((unsigned long long)__double_as_longlong(mag) & ~63ull) |
                                       (unsigned long long)(63 - i));
                    const unsigned long long best = __ockl_wfred_max_u64(key);
                    sh.fcol[buf][i] = v;
                    if (i == 0) {
                        const int p = 63 - (int)(best & 63ull);
                        sh.piv[buf] = p;
                        sh.perm[k] = p;
                    }
                }
                __syncthreads();
                const int p = sh.piv[buf];
                const double2 pv = sh.fcol[buf][p];
                const double2 fk = sh.fcol[buf][i];
                const double den = pv.x * pv.x + pv.y * pv.y;
                if (threadIdx.x == 0 && !(den > 0.0 && isfinite(den))) atomicOr(err, 1);
                const double2 inv = sel(den > 0.0, cmk<double2>(pv.x / den, -pv.y / den),
                                        cmk<double2>(0.0, 0.0));
                const double2 f = sel(i == p, cmk<double2>(0.0, 0.0), cmul(fk, inv));
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const double Rx = readlane_f64(M[r].x, p), Ry = readlane_f64(M[r].y, p);
                    M[r].x = fma(-f.x, Rx, fma(f.y, Ry, M[r].x));
                    M[r].y = fma(-f.x, Ry, fma(-f.y, Rx, M[r].y));
                }
                if (g == gg) {
                    M[0] = sel(i == p, cmk<double2>(1.0, 0.0), cmk<double2>(-f.x, -f.y));
                }
                if (i == p) {
                    used = true;
                    my_step = k;
                    my_inv = inv;
                }
            }
        }
        // rotate: the next four columns come to M[0]
        const double2 m0 = M[0];
#pragma unroll
        for (int r = 0; r < 15; ++r) M[r] = M[r + 1];
        M[15] = m0;
        ++rot;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int j = g + 4 * ((r + rot) & 15);
        const int pj = j < W ? sh.perm[j] : j;
        const double2 v = cmul(M[r], my_inv);
        dst[(size_t)pj * WP + my_step] = v;
        if (dst32) dst32[(size_t)pj * WP + my_step] = make_float2((float)v.x, (float)v.y);
    }
    __syncthreads();
}

}  // namespace gjr
}  // namespace helm

// Gauss-Jordan inversion of a 64 x 64 complex block held in registers (FP64) and a
// 64 x 64 complex block product on FP64 MFMA, shared by the strip factorisation (2-D) and
// the complex64 slab factorisation (3-D), where they invert the diagonal blocks.
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
    double nrm[2][4];        // per wave: largest column 1-norm of the block, of its inverse
};

// A block whose 1-norm condition estimate ||S||_1 ||S^-1||_1 exceeds this is numerically
// singular in FP64 (its inverse has no correct digit): the factorisation reports it
constexpr double GJ_COND_MAX = 1e13;

// sum over the 64 lanes of a wavefront (butterfly, every lane gets the sum)
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// largest column 1-norm over this wave's 16 register columns (rows i >= W are zero)
__device__ inline double wave_colnorm_max(const double2 (&M)[16]) {
    double best = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) best = fmax(best, wave_sum(sqrt(M[r].x * M[r].x + M[r].y * M[r].y)));
    return best;
}

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
// that dst can be read back by the workgroup.  Sets bit 1 of err when a pivot is zero or not
// finite, bit 2 when the 1-norm condition estimate exceeds GJ_COND_MAX.
__device__ inline void gj_invert_store(double2 (&M)[16], int W, GJShared& sh, double2* __restrict__ dst,
                                float2* __restrict__ dst32, int* err) {
    const int i = threadIdx.x & (WP - 1), g = threadIdx.x >> 6;
    bool used = i >= W;
    int my_step = i;                               // rows beyond W keep their position
    double2 my_inv = cmk<double2>(1.0, 0.0);
    int rot = 0;                                   // rotations done: M[r] holds column g + 4 (r + rot)
    {
        const double cn = wave_colnorm_max(M);
        if ((threadIdx.x & 63) == 0) sh.nrm[0][g] = cn;
    }
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
    double2 out[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int j = g + 4 * ((r + rot) & 15);
        const int pj = j < W ? sh.perm[j] : j;
        const double2 v = cmul(M[r], my_inv);
        out[r] = j < W ? v : cmk<double2>(0.0, 0.0);
        dst[(size_t)pj * WP + my_step] = v;
        if (dst32) dst32[(size_t)pj * WP + my_step] = make_float2((float)v.x, (float)v.y);
    }
    // permuting rows and columns leaves the set of column 1-norms unchanged: the largest
    // over the stored array is ||S^-1||_1 (the identity outside the leading block excluded)
    {
        const double cn = wave_colnorm_max(out);
        if ((threadIdx.x & 63) == 0) sh.nrm[1][g] = cn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < 4; ++q) { a = fmax(a, sh.nrm[0][q]); b = fmax(b, sh.nrm[1][q]); }
        if (!(a * b <= GJ_COND_MAX)) atomicOr(err, 2);
    }
}


// C = alpha * A * B (+ D) on v_mfma_f64_16x16x4f64: full WP x WP, column-major with leading
// dimensions, operands in LDS or global memory, C may alias A, B or D.  Wave w computes rows
// 16 w .. 16 w + 15 in four 16-column tiles; a complex product is four real ones.  Lane
// layout (one 16x16x4 block of doubles): A[l % 16][l / 16], B[l / 16][l % 16] and
// C[l / 16 + 4 j][l % 16] in component j (rows interleaved by 4, unlike the FP32 block).
typedef double md4 __attribute__((ext_vector_type(4)));

__device__ __attribute__((always_inline)) inline void gemm64_mfma(double2* C, int ldc, const double2* A, int lda, const double2* B, int ldb,
                            double2 alpha, const double2* D, int ldd) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, n = lane & 15, q4 = lane >> 4;
    double2 av[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) av[s] = A[(16 * w + n) + (size_t)(4 * s + q4) * lda];
    md4 cr[4], ci[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) { cr[tt] = md4{0.0, 0.0, 0.0, 0.0}; ci[tt] = cr[tt]; }
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        double2 bv[4];
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) bv[tt] = B[(4 * s + q4) + (size_t)(16 * tt + n) * ldb];
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
            cr[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s].x, bv[tt].x, cr[tt], 0, 0, 0);
            ci[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s].x, bv[tt].y, ci[tt], 0, 0, 0);
        }
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
            cr[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[s].y, bv[tt].y, cr[tt], 0, 0, 0);
            ci[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s].y, bv[tt].x, ci[tt], 0, 0, 0);
        }
    }
    double2 v[4][4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double2 x = cmul(alpha, cmk<double2>(cr[tt][j], ci[tt][j]));
            if (D) x = cadd(x, D[(16 * w + q4 + 4 * j) + (size_t)(16 * tt + n) * ldd]);
            v[tt][j] = x;
        }
    __syncthreads();
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int j = 0; j < 4; ++j) C[(16 * w + q4 + 4 * j) + (size_t)(16 * tt + n) * ldc] = v[tt][j];
    __syncthreads();
}

}  // namespace gjr
}  // namespace helm

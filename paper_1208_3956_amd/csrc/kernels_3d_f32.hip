// Complex64 slab factorisation of the mixed-precision 3-D path (the same block recursion
// along y as the FP64 one, Sec. 2.2 with the 7-point stencil):
//     S_0 = T_0,  S_l = T_l - c_l b_{l-1} G_{l-1},  G_l = S_l^{-1}.
// Each S_l is built over its own slot of the stored factor and inverted in place by
// blocked Gauss-Jordan elimination with pivoting only inside the 64 x 64 diagonal blocks:
// for the column block K,
//     P = A_KK^{-1}                                   (register Gauss-Jordan, FP64)
//     C = A(:, K) - E_K,   R = P [A(K, :) with A_KK := I]
//     A := A_mod - C R,    A_mod = A with the column block K replaced by E_K,
// which leaves A_KK = P, A(K, J) = P A(K, J), A(I, K) = -A(I, K) P and
// A(I, J) -= A(I, K) P A(K, J): one step of block Gauss-Jordan.  After the last block A
// holds S^{-1} with no permutation to undo.  The rows of block K are written as R
// directly rather than through the product (in FP32 that form would cancel to an error of
// order eps cond(A_KK)).  The update is a rank-64 complex GEMM on
// v_mfma_f32_16x16x4f32 with three real products per complex one (Gauss's form),
// accumulated in FP32.
// Without a search over the whole column the elimination relies on well-conditioned
// diagonal blocks: every inverted block's 1-norm condition number is checked, and the
// factorisation reports it (err bit 2) so that the caller can redo the slab factor with
// the FP64 Gauss-Jordan with partial pivoting over the whole column.
#include "helm_internal.hpp"
#include "gj_register.hpp"

namespace helm {

namespace {

using namespace gjr;

typedef float mf4 __attribute__((ext_vector_type(4)));

constexpr double COND_MAX = 1e6;   // largest accepted 1-norm condition of a diagonal block
// per-slab strides of the work arrays (the same for 64- and 128-wide blocks, so that slab
// groups on different streams never share a region)
constexpr size_t WSTR = 8 * (size_t)BLK;   // FP64 scratch blocks
constexpr size_t PSTR = 128 * 128;         // P
__host__ __device__ inline size_t cstr(int Bp) { return (size_t)128 * Bp; }   // C and R

// S_l = T_l - c_l b_{l-1} G_{l-1} into the plane-l slot of every slab (identity on the
// padding); G_{l-1} is the previous plane's slot (already inverted).  T in FP64, rounded.
__global__ void __launch_bounds__(256) k3f_build_S(Fac3Args a, int l, float2* __restrict__ F, size_t stride,
                                                  int s0) {
    const int s = s0 + blockIdx.y;
    const size_t BB = (size_t)a.Bp * a.Bp;
    const int W = a.sW[s], B = W * a.Nz;
    float2* S = F + s * stride + (size_t)l * BB;
    const float2* Gp = l > 0 ? S - BB : nullptr;
    double2 cb = make_double2(0.0, 0.0);
    if (l > 0) cb = cmul(a.cy[l], a.by[l - 1]);
    const double2 ydiag = cmul(a.ay[l], cadd(a.ayh[l + 1], a.ayh[l]));
    const double2* sax = a.sax + (size_t)s * WP;
    const double2* saxh = a.saxh + (size_t)s * (WP + 1);
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < BB; e += (size_t)gridDim.x * blockDim.x) {
        const int col = (int)(e / a.Bp), row = (int)(e % a.Bp);
        double2 v = make_double2(0.0, 0.0);
        if (row < B && col < B) {
            if (l > 0) {
                const float2 gp = Gp[e];
                v = cmk<double2>(-(cb.x * gp.x - cb.y * gp.y), -(cb.x * gp.y + cb.y * gp.x));
            }
            const int xr = row % W, zr = row / W, xc = col % W, zc = col / W;
            double2 t = make_double2(0.0, 0.0);
            if (row == col) {
                const double2 xd = cmul(sax[xr], cadd(saxh[xr + 1], saxh[xr]));
                const double2 zd = cmul(a.az[zr], cadd(a.azh[zr + 1], a.azh[zr]));
                t = cadd(cadd(xd, ydiag), zd);
                t.x *= a.ih2; t.y *= a.ih2;
                const int gx = a.scol[(size_t)s * WP + xr];
                t.x -= a.k2[((size_t)zr * a.Ny + l) * a.Nx + gx];
            } else if (zr == zc && (xc == xr + 1 || xc == xr - 1)) {
                t = cmul(sax[xr], xc == xr + 1 ? saxh[xr + 1] : saxh[xr]);
                t.x *= -a.ih2; t.y *= -a.ih2;
            } else if (xr == xc && (zc == zr + 1 || zc == zr - 1)) {
                t = cmul(a.az[zr], zc == zr + 1 ? a.azh[zr + 1] : a.azh[zr]);
                t.x *= -a.ih2; t.y *= -a.ih2;
            }
            v = cadd(v, t);
        } else if (row == col) {
            v = make_double2(1.0, 0.0);
        }
        S[e] = make_float2((float)v.x, (float)v.y);
    }
}

// P = A_KK^{-1} for the diagonal block at k0 of every slab (one workgroup per slab, the
// block in registers, FP64), stored column-major (leading dimension 64) in FP64 and
// complex64.  err bit 1: zero or non-finite pivot; bit 2: 1-norm condition above COND_MAX.
__global__ void __launch_bounds__(256) k3f_diag_inv(const float2* __restrict__ F, size_t stride, int l, int Bp,
                                                   int k0, double2* __restrict__ Pd, float2* __restrict__ Pf,
                                                   int* __restrict__ err, int s0) {
    __shared__ GJShared sh;
    __shared__ double na[4][64], np[4][64];
    const int s = s0 + blockIdx.x;
    const float2* A = F + s * stride + (size_t)l * Bp * Bp;
    const int i = threadIdx.x & 63, g = threadIdx.x >> 6;
    double2 M[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const float2 v = A[(size_t)(k0 + g + 4 * r) * Bp + k0 + i];
        M[r] = make_double2(v.x, v.y);
    }
    double2* pd = Pd + (size_t)s * WSTR;
    gj_invert_store(M, WP, sh, pd, Pf + (size_t)s * PSTR, err);
    {
        // column sums of |A_KK| and |P|: thread (column c, quarter h) sums 16 rows
        const int c = threadIdx.x & 63, h = threadIdx.x >> 6;
        double sa = 0.0, sp = 0.0;
#pragma unroll 4
        for (int r = 16 * h; r < 16 * h + 16; ++r) {
            const float2 v = A[(size_t)(k0 + c) * Bp + k0 + r];
            sa += sqrt((double)v.x * v.x + (double)v.y * v.y);
            const double2 p = pd[(size_t)c * WP + r];
            sp += sqrt(p.x * p.x + p.y * p.y);
        }
        na[h][c] = sa;
        np[h][c] = sp;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        // the maxima over the columns by one wave
        const int c = threadIdx.x;
        double ma = na[0][c] + na[1][c] + na[2][c] + na[3][c];
        double mp = np[0][c] + np[1][c] + np[2][c] + np[3][c];
        for (int off = 32; off > 0; off >>= 1) {
            ma = fmax(ma, __shfl_xor(ma, off));
            mp = fmax(mp, __shfl_xor(mp, off));
        }
        if (c == 0 && !(ma * mp <= COND_MAX)) atomicOr(err, 2);
    }
}

// P = A_KK^{-1} for a 128 x 128 diagonal block from its 64 x 64 blocks [A11 A12; A21 A22]:
//     P11 = A11^{-1},  S = A22 - A21 P11 A12,  P22 = S^{-1},
//     P12 = -P11 A12 P22,  P21 = -P22 A21 P11,  P11 <- P11 - P12 A21 P11
// (pivoting inside the two 64 x 64 inverses), in FP64, one workgroup per slab, with eight
// 64 x 64 scratch blocks per slab in global memory; P is stored complex64, column-major
// (leading dimension 128).  err bits as in the 64-wide kernel.
__global__ void __launch_bounds__(256) k3f_diag_inv128(const float2* __restrict__ F, size_t stride, int l, int Bp,
                                                      int k0, double2* __restrict__ Wd, float2* __restrict__ Pf,
                                                      int* __restrict__ err, int s0) {
    __shared__ GJShared sh;
    __shared__ double na[2][128], np[2][128];
    const int s = s0 + blockIdx.x, t = threadIdx.x;
    const float2* A = F + s * stride + (size_t)l * Bp * Bp;
    double2* W = Wd + (size_t)s * WSTR;
    double2 *A12 = W, *A21 = W + BLK, *A22 = W + 2 * BLK, *P11 = W + 3 * BLK;
    double2 *T1 = W + 4 * BLK, *P22 = W + 5 * BLK, *T2 = W + 6 * BLK, *P12 = W + 7 * BLK;
    auto at = [&](int r, int c) {
        const float2 v = A[(size_t)(k0 + c) * Bp + k0 + r];
        return make_double2(v.x, v.y);
    };
    for (int e = t; e < BLK; e += 256) {
        const int r = e % WP, c = e / WP;
        A12[e] = at(r, 64 + c);
        A21[e] = at(64 + r, c);
        A22[e] = at(64 + r, 64 + c);
    }
    const int i = t & 63, g = t >> 6;
    const double2 one = make_double2(1.0, 0.0), mone = make_double2(-1.0, 0.0);
    double2 M[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) M[r] = at(i, g + 4 * r);
    gj_invert_store(M, WP, sh, P11, nullptr, err);                 // ends with a barrier
    gemm64_mfma(T1, WP, P11, WP, A12, WP, one, nullptr, 0);        // T1 = P11 A12
    gemm64_mfma(A22, WP, A21, WP, T1, WP, mone, A22, WP);          // S = A22 - A21 T1
#pragma unroll
    for (int r = 0; r < 16; ++r) M[r] = A22[(size_t)(g + 4 * r) * WP + i];
    gj_invert_store(M, WP, sh, P22, nullptr, err);
    gemm64_mfma(P12, WP, T1, WP, P22, WP, mone, nullptr, 0);       // P12 = -T1 P22
    gemm64_mfma(T2, WP, A21, WP, P11, WP, one, nullptr, 0);        // T2 = A21 P11
    gemm64_mfma(A21, WP, P22, WP, T2, WP, mone, nullptr, 0);       // P21 = -P22 T2 (over A21)
    gemm64_mfma(P11, WP, P12, WP, T2, WP, mone, P11, WP);          // P11 = P11 - P12 T2
    float2* P = Pf + (size_t)s * PSTR;
    for (int e = t; e < 128 * 128; e += 256) {
        const int r = e % 128, c = e / 128;
        const double2* src = r < 64 ? (c < 64 ? P11 : P12) : (c < 64 ? A21 : P22);
        const double2 v = src[(size_t)(c & 63) * WP + (r & 63)];
        P[e] = make_float2((float)v.x, (float)v.y);
    }
    __syncthreads();
    {
        // column sums of |A_KK| and |P|: thread (column c, half h) sums 64 rows
        const int c = t & 127, h = t >> 7;
        double sa = 0.0, sp = 0.0;
#pragma unroll 4
        for (int r = 64 * h; r < 64 * h + 64; ++r) {
            const double2 v = at(r, c);
            sa += sqrt(v.x * v.x + v.y * v.y);
            const float2 q = P[(size_t)c * 128 + r];
            sp += sqrt((double)q.x * q.x + (double)q.y * q.y);
        }
        na[h][c] = sa;
        np[h][c] = sp;
    }
    __syncthreads();
    if (t < 64) {
        double ma = fmax(na[0][t] + na[1][t], na[0][t + 64] + na[1][t + 64]);
        double mp = fmax(np[0][t] + np[1][t], np[0][t + 64] + np[1][t + 64]);
        for (int off = 32; off > 0; off >>= 1) {
            ma = fmax(ma, __shfl_xor(ma, off));
            mp = fmax(mp, __shfl_xor(mp, off));
        }
        if (t == 0 && !(ma * mp <= COND_MAX)) atomicOr(err, 2);
    }
}

// The operands of the update for the column block K = k0 .. k0 + NB - 1 (grid: 64-column
// tiles x slabs):
//   C(i, k) = A(i, k0 + k) - [i = k0 + k]     rows of tile jt,  stored Cb[s][k][Bp]
//   R(k, j) = sum_m P(k, m) A(k0 + m, j)      columns of tile jt, R(:, K) = P, Rb[s][k][Bp]
// P is NB x NB, column-major (leading dimension NB).  The NB x 64 x NB product runs on
// v_mfma_f32_16x16x4f32: wave w computes rows NB/4 w .. of R for the tile's 64 columns, P
// read in lane layout from global memory, the A block from LDS (staged column by column).
template <int NB>
__global__ void __launch_bounds__(256) k3f_rc(const float2* __restrict__ F, size_t stride, int l, int Bp, int k0,
                                             const float2* __restrict__ Pf, float2* __restrict__ Cb,
                                             float2* __restrict__ Rb, int s0) {
    constexpr int RW = NB / 64;        // 16-row MFMA tiles per wave
    __shared__ float2 As[64][NB + 1];  // As[j][m] = A(k0 + m, J0 + j)
    const int s = s0 + blockIdx.y, J0 = blockIdx.x * 64, t = threadIdx.x;
    const float2* A = F + s * stride + (size_t)l * Bp * Bp;
    float2* cb = Cb + (size_t)s * cstr(Bp);
    float2* rb = Rb + (size_t)s * cstr(Bp);
    const float2* P = Pf + (size_t)s * PSTR;
    // C rows of this tile
    for (int e = t; e < NB * 64; e += 256) {
        const int k = e / 64, ii = e % 64, i = J0 + ii;
        float2 v = A[(size_t)(k0 + k) * Bp + i];
        if (i == k0 + k) v.x -= 1.0f;
        cb[(size_t)k * Bp + i] = v;
    }
    if (J0 >= k0 && J0 < k0 + NB) {
        for (int e = t; e < NB * 64; e += 256) {
            const int k = e / 64, jj = e % 64;
            rb[(size_t)k * Bp + J0 + jj] = P[(size_t)(J0 - k0 + jj) * NB + k];
        }
        return;
    }
    for (int e = t; e < NB * 64; e += 256) {
        const int jj = e / NB, mm = e % NB;
        As[jj][mm] = A[(size_t)(J0 + jj) * Bp + k0 + mm];
    }
    __syncthreads();
    const int lane = t & 63, w = t >> 6, n = lane & 15, q4 = lane >> 4;
    mf4 re[RW][4], im[RW][4];
#pragma unroll
    for (int ra = 0; ra < RW; ++ra)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) { re[ra][jb] = mf4{0.f, 0.f, 0.f, 0.f}; im[ra][jb] = re[ra][jb]; }
    const float2* pp = P + (size_t)q4 * NB + 16 * RW * w + n;     // P(16 (RW w + ra) + n, 4 ks + q4)
#pragma unroll 2
    for (int ks = 0; ks < NB / 4; ++ks) {
        float2 a[RW];
#pragma unroll
        for (int ra = 0; ra < RW; ++ra) a[ra] = pp[(size_t)4 * ks * NB + 16 * ra];
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
            const float2 b = As[16 * jb + n][4 * ks + q4];
#pragma unroll
            for (int ra = 0; ra < RW; ++ra) {
                re[ra][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ra].x, b.x, re[ra][jb], 0, 0, 0);
                im[ra][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ra].x, b.y, im[ra][jb], 0, 0, 0);
                re[ra][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[ra].y, b.y, re[ra][jb], 0, 0, 0);
                im[ra][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ra].y, b.x, im[ra][jb], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int ra = 0; ra < RW; ++ra)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                rb[(size_t)(16 * (RW * w + ra) + 4 * q4 + j) * Bp + J0 + 16 * jb + n] =
                    make_float2(re[ra][jb][j], im[ra][jb][j]);
}

// A := A_mod - C R on every 64 x 64 tile of every slab.  The tiles are spread over the
// eight XCDs in contiguous runs of the slab-major, column-major tile order (a run covers
// whole columns of one or two slabs, so the C panel and the R columns a run reads stay in
// that XCD's L2).  Wave w computes the 32 x 32 quadrant (w & 1, w >> 1) as 2 x 2 MFMA
// tiles; operands are read straight from global memory in the MFMA lane layout (A operand
// C(l % 16, l / 16), B operand R(l / 16, l % 16), accumulator rows 4 (l / 16) + j, column
// l % 16), one k-step ahead.
template <int NB>
__global__ void __launch_bounds__(256) k3f_update(float2* __restrict__ F, size_t stride, int l, int Bp, int k0,
                                                 int ns, const float2* __restrict__ Cb,
                                                 const float2* __restrict__ Rb, int s0) {
    const int nb = Bp / 64, nt = nb * nb;
    const int total = ns * nt, per = (total + 7) / 8;
    const int gi = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (gi >= total) return;
    const int s = s0 + gi / nt, tt = gi % nt, it = tt % nb, jt = tt / nb;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, n = lane & 15, q4 = lane >> 4;
    const int I0 = it * 64 + 32 * (w & 1), J0 = jt * 64 + 32 * (w >> 1);
    float2* A = F + s * stride + (size_t)l * Bp * Bp;
    const float2* cp = Cb + (size_t)s * cstr(Bp) + (size_t)q4 * Bp + I0 + n;
    const float2* rp = Rb + (size_t)s * cstr(Bp) + (size_t)q4 * Bp + J0 + n;
    const bool kcol = jt * 64 >= k0 && jt * 64 < k0 + NB;
    if (it * 64 >= k0 && it * 64 < k0 + NB) {
        // the rows of block K become R(:, J) = P A(K, J): written directly, since forming
        // them as A(K, J) - (A_KK - I) R(:, J) would cancel A(K, J) against A_KK P A(K, J)
        // and leave an FP32 error of order eps cond(A_KK)
        const float2* rr = Rb + (size_t)s * cstr(Bp);
#pragma unroll
        for (int ia = 0; ia < 2; ++ia)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb) {
                const int col = J0 + 16 * jb + n;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = I0 + 16 * ia + 4 * q4 + j;
                    A[(size_t)col * Bp + row] = rr[(size_t)(row - k0) * Bp + col];
                }
            }
        return;
    }
    // complex products by three real ones (x1 = -sum Cr Rr, x2 = sum Ci Ri,
    // x3 = -sum (Cr + Ci)(Rr + Ri)):  Re = A.r + x1 + x2,  Im = A.i + x3 - x1 + x2
    float2 av[2][2][4];
#pragma unroll
    for (int ia = 0; ia < 2; ++ia)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
            const int col = J0 + 16 * jb + n;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = I0 + 16 * ia + 4 * q4 + j;
                av[ia][jb][j] = kcol ? make_float2(row == col ? 1.f : 0.f, 0.f) : A[(size_t)col * Bp + row];
            }
        }
    mf4 x1[2][2], x2[2][2], x3[2][2];
#pragma unroll
    for (int ia = 0; ia < 2; ++ia)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
            x1[ia][jb] = mf4{0.f, 0.f, 0.f, 0.f};
            x2[ia][jb] = x1[ia][jb];
            x3[ia][jb] = x1[ia][jb];
        }
    float2 c[2], r[2], cn[2], rn[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) { c[u] = cp[16 * u]; r[u] = rp[16 * u]; }
    for (int kb = 0; kb < NB / 4; ++kb) {
        const size_t nx = (size_t)(kb + 1 < NB / 4 ? kb + 1 : kb) * 4 * Bp;
#pragma unroll
        for (int u = 0; u < 2; ++u) { cn[u] = cp[nx + 16 * u]; rn[u] = rp[nx + 16 * u]; }
        float cs[2], rs[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) { cs[u] = c[u].x + c[u].y; rs[u] = r[u].x + r[u].y; }
#pragma unroll
        for (int ia = 0; ia < 2; ++ia)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb) {
                x1[ia][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(-c[ia].x, r[jb].x, x1[ia][jb], 0, 0, 0);
                x2[ia][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(c[ia].y, r[jb].y, x2[ia][jb], 0, 0, 0);
                x3[ia][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(-cs[ia], rs[jb], x3[ia][jb], 0, 0, 0);
            }
#pragma unroll
        for (int u = 0; u < 2; ++u) { c[u] = cn[u]; r[u] = rn[u]; }
    }
#pragma unroll
    for (int ia = 0; ia < 2; ++ia)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
            const int col = J0 + 16 * jb + n;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = I0 + 16 * ia + 4 * q4 + j;
                const float2 a0 = av[ia][jb][j];
                const float p1 = x1[ia][jb][j], p2 = x2[ia][jb][j], p3 = x3[ia][jb][j];
                A[(size_t)col * Bp + row] = make_float2(a0.x + p1 + p2, a0.y + p3 - p1 + p2);
            }
        }
}

}  // namespace

size_t factor3_f32_work_bytes(int J, int Bp) {
    // per slab: eight FP64 64 x 64 scratch blocks (the 64-wide inverse uses the first),
    // P (complex64, up to 128 x 128), C and R (up to 128 x Bp each)
    return (size_t)J * (WSTR * sizeof(double2) + PSTR * sizeof(float2) + 2 * cstr(Bp) * sizeof(float2));
}

// One plane of the slabs s0 .. s0 + ns - 1: column blocks of 128 (a last block of 64 when
// Bp is an odd multiple of 64).  A 128-wide block halves the passes of the update over the
// matrices (the update is bound by HBM and MFMA about equally at 64).
hipError_t launch_factor3_plane_f32(const Fac3Args& a, int l, float2* F, size_t stride, void* work, int* err,
                                    hipStream_t st, int s0, int ns) {
    const size_t BB = (size_t)a.Bp * a.Bp;
    double2* Wd = static_cast<double2*>(work);
    float2* Pf = reinterpret_cast<float2*>(Wd + (size_t)a.J * WSTR);
    float2* Cb = Pf + (size_t)a.J * PSTR;
    float2* Rb = Cb + (size_t)a.J * cstr(a.Bp);
    const unsigned nbs = (unsigned)std::min<size_t>((BB + 255) / 256, 4096);
    hipLaunchKernelGGL(k3f_build_S, dim3(nbs, ns), dim3(256), 0, st, a, l, F, stride, s0);
    const int nb = a.Bp / 64;
    const int total = ns * nb * nb, per = (total + 7) / 8;
    for (int k0 = 0; k0 < a.Bp;) {
        if (k0 + 128 <= a.Bp) {
            hipLaunchKernelGGL(k3f_diag_inv128, dim3(ns), dim3(256), 0, st, F, stride, l, a.Bp, k0, Wd, Pf, err, s0);
            hipLaunchKernelGGL(k3f_rc<128>, dim3(nb, ns), dim3(256), 0, st, F, stride, l, a.Bp, k0, Pf, Cb, Rb, s0);
            hipLaunchKernelGGL(k3f_update<128>, dim3(8 * per), dim3(256), 0, st, F, stride, l, a.Bp, k0, ns, Cb, Rb,
                               s0);
            k0 += 128;
        } else {
            hipLaunchKernelGGL(k3f_diag_inv, dim3(ns), dim3(256), 0, st, F, stride, l, a.Bp, k0, Wd, Pf, err, s0);
            hipLaunchKernelGGL(k3f_rc<64>, dim3(nb, ns), dim3(256), 0, st, F, stride, l, a.Bp, k0, Pf, Cb, Rb, s0);
            hipLaunchKernelGGL(k3f_update<64>, dim3(8 * per), dim3(256), 0, st, F, stride, l, a.Bp, k0, ns, Cb, Rb,
                               s0);
            k0 += 64;
        }
    }
    return hipGetLastError();
}

}  // namespace helm

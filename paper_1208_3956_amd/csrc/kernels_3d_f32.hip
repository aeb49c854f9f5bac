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

constexpr int NBF = 64;            // block width
constexpr double COND_MAX = 1e6;   // largest accepted 1-norm condition of a diagonal block

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
    double2* pd = Pd + (size_t)s * BLK;
    gj_invert_store(M, WP, sh, pd, Pf + (size_t)s * BLK, err);
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

// The operands of the update for column block k0 (grid: column tiles x slabs):
//   C(i, k) = A(i, k0 + k) - [i = k0 + k]     rows of tile jt,  stored Cb[s][k][Bp]
//   R(k, j) = sum_m P(k, m) A(k0 + m, j)      columns of tile jt, R(:, K) = P, Rb[s][k][Bp]
// The 64 x 64 x 64 product runs on v_mfma_f32_16x16x4f32: wave w computes rows
// 16w .. 16w + 15 of R for the tile's 64 columns, P read in lane layout from global
// memory, the A block from LDS (staged column by column, coalesced).
__global__ void __launch_bounds__(256) k3f_rc(const float2* __restrict__ F, size_t stride, int l, int Bp, int k0,
                                             const float2* __restrict__ Pf, float2* __restrict__ Cb,
                                             float2* __restrict__ Rb, int s0) {
    __shared__ float2 As[64][65];      // As[j][m] = A(k0 + m, J0 + j)
    const int s = s0 + blockIdx.y, J0 = blockIdx.x * NBF, t = threadIdx.x;
    const float2* A = F + s * stride + (size_t)l * Bp * Bp;
    float2* cb = Cb + (size_t)s * NBF * Bp;
    float2* rb = Rb + (size_t)s * NBF * Bp;
    const float2* P = Pf + (size_t)s * BLK;
    // C rows of this tile
    for (int e = t; e < NBF * NBF; e += 256) {
        const int k = e / NBF, ii = e % NBF, i = J0 + ii;
        float2 v = A[(size_t)(k0 + k) * Bp + i];
        if (i == k0 + k) v.x -= 1.0f;
        cb[(size_t)k * Bp + i] = v;
    }
    if (J0 == k0) {
        for (int e = t; e < NBF * NBF; e += 256) {
            const int k = e / NBF, jj = e % NBF;
            rb[(size_t)k * Bp + J0 + jj] = P[(size_t)jj * WP + k];
        }
        return;
    }
    for (int e = t; e < NBF * NBF; e += 256) {
        const int jj = e / NBF, mm = e % NBF;
        As[jj][mm] = A[(size_t)(J0 + jj) * Bp + k0 + mm];
    }
    __syncthreads();
    const int lane = t & 63, w = t >> 6, n = lane & 15, q4 = lane >> 4;
    mf4 re[4], im[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) { re[jb] = mf4{0.f, 0.f, 0.f, 0.f}; im[jb] = re[jb]; }
    const float2* pp = P + (size_t)q4 * WP + 16 * w + n;     // P(16w + n, 4 ks + q4)
#pragma unroll 4
    for (int ks = 0; ks < NBF / 4; ++ks) {
        const float2 a = pp[(size_t)4 * ks * WP];
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
            const float2 b = As[16 * jb + n][4 * ks + q4];
            re[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, re[jb], 0, 0, 0);
            im[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.y, im[jb], 0, 0, 0);
            re[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, b.y, re[jb], 0, 0, 0);
            im[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.x, im[jb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            rb[(size_t)(16 * w + 4 * q4 + j) * Bp + J0 + 16 * jb + n] = make_float2(re[jb][j], im[jb][j]);
}

// A := A_mod - C R on every 64 x 64 tile of every slab.  The tiles are spread over the
// eight XCDs in contiguous runs of the slab-major, column-major tile order (a run covers
// whole columns of one or two slabs, so the C panel and the R columns a run reads stay in
// that XCD's L2).  Wave w computes the 32 x 32 quadrant (w & 1, w >> 1) as 2 x 2 MFMA
// tiles; operands are read straight from global memory in the MFMA lane layout (A operand
// C(l % 16, l / 16), B operand R(l / 16, l % 16), accumulator rows 4 (l / 16) + j, column
// l % 16), one k-step ahead.
__global__ void __launch_bounds__(256) k3f_update(float2* __restrict__ F, size_t stride, int l, int Bp, int k0,
                                                 int ns, const float2* __restrict__ Cb,
                                                 const float2* __restrict__ Rb, int s0) {
    const int nb = Bp / NBF, nt = nb * nb;
    const int total = ns * nt, per = (total + 7) / 8;
    const int gi = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (gi >= total) return;
    const int s = s0 + gi / nt, tt = gi % nt, it = tt % nb, jt = tt / nb;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, n = lane & 15, q4 = lane >> 4;
    const int I0 = it * NBF + 32 * (w & 1), J0 = jt * NBF + 32 * (w >> 1);
    float2* A = F + s * stride + (size_t)l * Bp * Bp;
    const float2* cp = Cb + (size_t)s * NBF * Bp + (size_t)q4 * Bp + I0 + n;
    const float2* rp = Rb + (size_t)s * NBF * Bp + (size_t)q4 * Bp + J0 + n;
    const bool kcol = jt * NBF == k0;
    if (it * NBF == k0) {
        // the rows of block K become R(:, J) = P A(K, J): written directly, since forming
        // them as A(K, J) - (A_KK - I) R(:, J) would cancel A(K, J) against A_KK P A(K, J)
        // and leave an FP32 error of order eps cond(A_KK)
        const float2* rr = Rb + (size_t)s * NBF * Bp;
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
    for (int kb = 0; kb < NBF / 4; ++kb) {
        const size_t nx = (size_t)(kb + 1 < NBF / 4 ? kb + 1 : kb) * 4 * Bp;
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
    // Pd (FP64) + Pf + Cb + Rb per slab
    return (size_t)J * (BLK * sizeof(double2) + BLK * sizeof(float2) + 2 * (size_t)NBF * Bp * sizeof(float2));
}

hipError_t launch_factor3_plane_f32(const Fac3Args& a, int l, float2* F, size_t stride, void* work, int* err,
                                    hipStream_t st, int s0, int ns) {
    const size_t BB = (size_t)a.Bp * a.Bp;
    double2* Pd = static_cast<double2*>(work);
    float2* Pf = reinterpret_cast<float2*>(Pd + (size_t)a.J * BLK);
    float2* Cb = Pf + (size_t)a.J * BLK;
    float2* Rb = Cb + (size_t)a.J * NBF * a.Bp;
    const unsigned nbs = (unsigned)std::min<size_t>((BB + 255) / 256, 4096);
    hipLaunchKernelGGL(k3f_build_S, dim3(nbs, ns), dim3(256), 0, st, a, l, F, stride, s0);
    const int nb = a.Bp / NBF;
    const int total = ns * nb * nb, per = (total + 7) / 8;
    for (int k0 = 0; k0 < a.Bp; k0 += NBF) {
        hipLaunchKernelGGL(k3f_diag_inv, dim3(ns), dim3(256), 0, st, F, stride, l, a.Bp, k0, Pd, Pf, err, s0);
        hipLaunchKernelGGL(k3f_rc, dim3(nb, ns), dim3(256), 0, st, F, stride, l, a.Bp, k0, Pf, Cb, Rb, s0);
        hipLaunchKernelGGL(k3f_update, dim3(8 * per), dim3(256), 0, st, F, stride, l, a.Bp, k0, ns, Cb, Rb, s0);
    }
    return hipGetLastError();
}

}  // namespace helm

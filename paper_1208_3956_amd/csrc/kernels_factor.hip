// Strip factorisation (the subdomain factorisation of Algorithm 1, Sec. 2.3).
//
// A padded strip operator A^(j) (Sec. 2.2, grid of eq. grid_A_j) ordered row by row in y
// is block tridiagonal: diagonal blocks T_l (W x W, tridiagonal in x: the x part of the
// PML stencil plus the y diagonal and -k^2), and off-diagonal blocks that are scalar
// multiples of the identity, c_l I (row l to row l-1) and b_l I (row l to row l+1),
// because the y-PML coefficients do not depend on x.
//
// The y rows are cut into chunks of m rows; the last row of every chunk but the last is
// a separator.  Per chunk (interior rows r0..r1-1), in FP64:
//   block LU       S_r0 = T_r0,  S_l = T_l - c_l b_{l-1} S_{l-1}^{-1},  G_l = S_l^{-1}
//   top spike      X~ = A_I^{-1} (coupling to the separator above) = c_r0 * A_I^{-1} E_first
//   bottom spike   Y~ = A_I^{-1} (coupling to the separator below) = b_{r1-1} * A_I^{-1} E_last
// and per strip the separators' block-tridiagonal Schur complement is factored by block
// LU (G'_c, K_c = G'_c L_c, U'_c = G'_c S^_{c,c+1}).  Storage per row l: three WP x WP blocks
// (slot 0: G or G', slot 1: X~ or K, slot 2: Y~ or U').
//
// Inverses are formed by Gauss-Jordan elimination with partial (row) pivoting, the matrix
// held in registers (one row per lane, the 64 columns split over the four waves).
#include "helm_internal.hpp"
#include "gj_register.hpp"

namespace helm {

namespace {

using namespace gjr;

constexpr int LDM = WP + 1;   // LDS leading dimension (bank spreading)
constexpr int NT = 256;

struct FactorArgs {
    double2* F;
    float2* F32;            // complex64 copy of every stored block (null: none)
    const double* k2;
    const double2* ay;
    const double2* ayh;
    const double2* cy;
    const double2* by;
    const double2* sax;
    const double2* saxh;
    const int* scol;
    const int* sW;
    // Robin subdomains (the comparison method of Sec. 4.4): [strip][row][2] terms added to
    // the diagonal of the first / last column of every row (null: PML pads)
    const double2* rob;
    int* err;
    int Nx, Ny, m, P;
    double inv_h2;
};

__device__ inline double2 ld_scaled(const double2* p, double2 s) { return cmul(*p, s); }

// Zero an LDS matrix and write the diagonal block T_l of strip s.
__device__ void build_T(double2* M, const FactorArgs& a, int s, int l, int W) {
    const int t = threadIdx.x;
    for (int idx = t; idx < WP * LDM; idx += NT) M[idx] = cmk<double2>(0.0, 0.0);
    __syncthreads();
    if (t < W) {
        const double2* sx = a.sax + (size_t)s * WP;
        const double2* sxh = a.saxh + (size_t)s * (WP + 1);
        const double2 axq = sx[t];
        const double2 e = sxh[t + 1], wv = sxh[t];
        const double2 ayl = a.ay[l];
        const double2 n = a.ayh[l + 1], so = a.ayh[l];
        double2 d = cmul(axq, cadd(e, wv));
        d = cadd(d, cmul(ayl, cadd(n, so)));
        d.x *= a.inv_h2; d.y *= a.inv_h2;
        d.x -= a.k2[(size_t)l * a.Nx + a.scol[(size_t)s * WP + t]];
        if (a.rob) {
            if (t == 0) d = cadd(d, a.rob[((size_t)s * a.Ny + l) * 2]);
            if (t == W - 1) d = cadd(d, a.rob[((size_t)s * a.Ny + l) * 2 + 1]);
        }
        M[t + t * LDM] = d;
        if (t + 1 < W) {
            double2 o = cmul(axq, e);
            M[t + (t + 1) * LDM] = cmk<double2>(-o.x * a.inv_h2, -o.y * a.inv_h2);
        }
        if (t >= 1) {
            double2 o = cmul(axq, wv);
            M[t + (t - 1) * LDM] = cmk<double2>(-o.x * a.inv_h2, -o.y * a.inv_h2);
        }
    }
    __syncthreads();
}


__device__ inline double2* slot(const FactorArgs& a, int s, int l, int sl) {
    return a.F + (((size_t)s * a.Ny + l) * NSLOT + sl) * BLK;
}
__device__ inline float2* slot32(const FactorArgs& a, int s, int l, int sl) {
    return a.F32 ? a.F32 + (((size_t)s * a.Ny + l) * NSLOT + sl) * BLK : nullptr;
}

// LDS (ld LDM) -> global (ld WP), optionally scaled; dst32 (if not null) gets the same
// block rounded to complex64.
__device__ void store_blk(double2* dst, float2* dst32, const double2* M, double2 scale) {
    for (int idx = threadIdx.x; idx < BLK; idx += NT) {
        const int i = idx & (WP - 1), k = idx / WP;
        const double2 v = cmul(M[i + k * LDM], scale);
        dst[idx] = v;
        if (dst32) dst32[idx] = make_float2((float)v.x, (float)v.y);
    }
}
__device__ void load_blk(double2* M, const double2* src) {
    for (int idx = threadIdx.x; idx < BLK; idx += NT) {
        const int i = idx & (WP - 1), k = idx / WP;
        M[i + k * LDM] = src[idx];
    }
}

// Block LU of the chunk interior, G_l = (T_l - c_l b_{l-1} G_{l-1})^{-1}, one chunk per
// workgroup, the matrices in registers (layout of gj_invert_store).  G_{l-1} is read back
// from its slot in natural order.
__global__ void __launch_bounds__(NT) k_factor_chunks(FactorArgs a) {
    __shared__ GJShared sh;
    const int c = blockIdx.x, s = blockIdx.y;
    const int W = a.sW[s];
    const int r0 = c * a.m;
    const int r1 = (c < a.P - 1) ? c * a.m + a.m - 1 : a.Ny;
    const int i = threadIdx.x & (WP - 1), g = threadIdx.x >> 6;
    // the x part of row i of T_l (the same on every row l of the strip)
    double2 xd = cmk<double2>(0.0, 0.0), xup = xd, xlo = xd;
    int col = 0;
    if (i < W) {
        const double2 axq = a.sax[(size_t)s * WP + i];
        const double2 e = a.saxh[(size_t)s * (WP + 1) + i + 1], wv = a.saxh[(size_t)s * (WP + 1) + i];
        xd = cmul(axq, cadd(e, wv));
        const double2 o = cmul(axq, e), q = cmul(axq, wv);
        xup = cmk<double2>(-o.x * a.inv_h2, -o.y * a.inv_h2);
        xlo = cmk<double2>(-q.x * a.inv_h2, -q.y * a.inv_h2);
        col = a.scol[(size_t)s * WP + i];
    }
    double2 M[16];
    for (int l = r0; l < r1; ++l) {
        double2 d = cadd(xd, cmul(a.ay[l], cadd(a.ayh[l + 1], a.ayh[l])));
        d.x *= a.inv_h2; d.y *= a.inv_h2;
        d.x -= a.k2[(size_t)l * a.Nx + col];
        if (a.rob) {
            if (i == 0) d = cadd(d, a.rob[((size_t)s * a.Ny + l) * 2]);
            if (i == W - 1) d = cadd(d, a.rob[((size_t)s * a.Ny + l) * 2 + 1]);
        }
        const double2 cb = l > r0 ? cmul(a.cy[l], a.by[l - 1]) : cmk<double2>(0.0, 0.0);
        const double2* Gp = slot(a, s, l > r0 ? l - 1 : l, 0);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int j = g + 4 * r;
            double2 v = cmk<double2>(0.0, 0.0);
            if (i < W && j < W) {
                v = sel(j == i, d, sel(j == i + 1, xup, sel(j == i - 1, xlo, v)));
                if (l > r0) v = csub(v, cmul(cb, Gp[(size_t)j * WP + i]));
            }
            M[r] = v;
        }
        gj_invert_store(M, W, sh, slot(a, s, l, 0), slot32(a, s, l, 0), a.err);
    }
}

// The two spikes of a chunk (blockIdx.z = 0: top, 1: bottom), after the inversions.
__global__ void __launch_bounds__(NT) k_factor_spikes(FactorArgs a) {
    __shared__ double2 bufA[WP * LDM];
    __shared__ double2 bufB[WP * LDM];
    const int c = blockIdx.x, s = blockIdx.y, side = blockIdx.z;
    const int r0 = c * a.m;
    const int r1 = (c < a.P - 1) ? c * a.m + a.m - 1 : a.Ny;
    const double2 one = cmk<double2>(1.0, 0.0);
    double2* Pm = bufA;
    double2* Cm = bufB;

    // ---- top spike: forward Z_r0 = G_r0, Z_l = -c_l G_l Z_{l-1}; backward
    //      X_l = Z_l - b_l G_l X_{l+1};  stored scaled by c_r0
    if (side == 0 && c > 0) {
        load_blk(Pm, slot(a, s, r0, 0));
        __syncthreads();
        store_blk(slot(a, s, r0, 1), slot32(a, s, r0, 1), Pm, one);
        for (int l = r0 + 1; l < r1; ++l) {
            const double2 cl = a.cy[l];
            gemm64_mfma(Cm, LDM, slot(a, s, l, 0), WP, Pm, LDM, cmk<double2>(-cl.x, -cl.y), nullptr, 0);
            store_blk(slot(a, s, l, 1), slot32(a, s, l, 1), Cm, one);
            double2* tmp = Pm; Pm = Cm; Cm = tmp;
        }
        __threadfence();
        __syncthreads();
        const double2 ctop = a.cy[r0];
        store_blk(slot(a, s, r1 - 1, 1), slot32(a, s, r1 - 1, 1), Pm, ctop);
        for (int l = r1 - 2; l >= r0; --l) {
            const double2 bl = a.by[l];
            gemm64_mfma(Cm, LDM, slot(a, s, l, 0), WP, Pm, LDM, cmk<double2>(-bl.x, -bl.y),
                   slot(a, s, l, 1), WP);
            store_blk(slot(a, s, l, 1), slot32(a, s, l, 1), Cm, ctop);
            double2* tmp = Pm; Pm = Cm; Cm = tmp;
        }
        __syncthreads();
    }

    // ---- bottom spike: Y_{r1-1} = G_{r1-1}, Y_l = -b_l G_l Y_{l+1}; stored scaled by b_{r1-1}
    if (side == 1 && c < a.P - 1) {
        const double2 bbot = a.by[r1 - 1];
        load_blk(Pm, slot(a, s, r1 - 1, 0));
        __syncthreads();
        store_blk(slot(a, s, r1 - 1, 2), slot32(a, s, r1 - 1, 2), Pm, bbot);
        for (int l = r1 - 2; l >= r0; --l) {
            const double2 bl = a.by[l];
            gemm64_mfma(Cm, LDM, slot(a, s, l, 0), WP, Pm, LDM, cmk<double2>(-bl.x, -bl.y), nullptr, 0);
            store_blk(slot(a, s, l, 2), slot32(a, s, l, 2), Cm, bbot);
            double2* tmp = Pm; Pm = Cm; Cm = tmp;
        }
    }
}

// Block LU of the separators' Schur complement, one workgroup per strip, sequential over
// separators c = 0..P-2 (row s = sep(c)):
//   S^_cc      = T_s - c_s Y~^(c)_{s-1} - b_s X~^(c+1)_{s+1}
//   S^_{c,c-1} = -c_s X~^(c)_{s-1}           (stored as L_c in slot 1)
//   S^_{c,c+1} = -b_s Y~^(c+1)_{s+1}
//   S'_c = S^_cc - L_c U'_{c-1},  G'_c = S'_c^{-1} (slot 0),  K_c = G'_c L_c (slot 1),
//   U'_c = G'_c S^_{c,c+1} (slot 2)
__global__ void __launch_bounds__(NT) k_factor_separators(FactorArgs a) {
    __shared__ double2 Am[WP * LDM];
    __shared__ double2 Bm[WP * LDM];
    __shared__ GJShared sh;
    const int s = blockIdx.x;
    const int W = a.sW[s];
    const double2 one = cmk<double2>(1.0, 0.0);
    for (int c = 0; c + 1 < a.P; ++c) {
        const int r = c * a.m + a.m - 1;
        build_T(Bm, a, s, r, W);
        const double2 cs = a.cy[r], bs = a.by[r];
        {
            const double2* Yc = slot(a, s, r - 1, 2);
            const double2* Xn = slot(a, s, r + 1, 1);
            for (int idx = threadIdx.x; idx < BLK; idx += NT) {
                const int i = idx & (WP - 1), k = idx / WP;
                double2 v = Bm[i + k * LDM];
                v = csub(v, cmul(cs, Yc[idx]));
                v = csub(v, cmul(bs, Xn[idx]));
                Bm[i + k * LDM] = v;
            }
        }
        __syncthreads();
        if (c >= 1) {
            // Bm = Bm - L_c U'_{c-1},  L_c = S^_{c,c-1} = -c_s X~^(c)_{s-1}
            gemm64_mfma(Bm, LDM, slot(a, s, r - 1, 1), WP, Am, LDM, cs, Bm, LDM);
        }
        {
            double2 M[16];
            const int i = threadIdx.x & (WP - 1), g = threadIdx.x >> 6;
#pragma unroll
            for (int q = 0; q < 16; ++q) M[q] = Bm[i + (g + 4 * q) * LDM];
            gj_invert_store(M, W, sh, slot(a, s, r, 0), slot32(a, s, r, 0), a.err);
        }
        const double2* Gp = slot(a, s, r, 0);
        if (c >= 1) {
            // K_c = G'_c L_c = -c_s G'_c X~^(c)_{s-1} replaces L_c in slot 1, so that the
            // forward separator recurrence is z'_c = G'_c r^_c - K_c z'_{c-1}
            gemm64_mfma(Am, LDM, Gp, WP, slot(a, s, r - 1, 1), WP, cmk<double2>(-cs.x, -cs.y), nullptr, 0);
            store_blk(slot(a, s, r, 1), slot32(a, s, r, 1), Am, one);
            __syncthreads();
        }
        if (c + 2 < a.P) {
            gemm64_mfma(Am, LDM, Gp, WP, slot(a, s, r + 1, 2), WP, cmk<double2>(-bs.x, -bs.y), nullptr, 0);
            store_blk(slot(a, s, r, 2), slot32(a, s, r, 2), Am, one);
            __syncthreads();
        }
    }
}

// Propagators of the two-level separator solve (grid: strips x groups x direction).
// Forward (group g >= 1, separators c0..c1): Phi_{c0} = -K_{c0}, Phi_c = -K_c Phi_{c-1}, so
// that z'_c = zeta_c + Phi_c z'_{c0-1} with zeta the group's own recurrence started from 0.
// Backward (group g <= G-2): Psi_{c1} = -U'_{c1}, Psi_c = -U'_c Psi_{c+1}, so that
// x_c = xi_c + Psi_c x_{c1+1}.
__global__ void __launch_bounds__(NT) k_factor_propagators(FactorArgs a, int q, int G, double2* __restrict__ Fs,
                                                           float2* __restrict__ Fs32) {
    __shared__ double2 Am[WP * LDM];
    __shared__ double2 Bm[WP * LDM];
    const int s = blockIdx.x, g = blockIdx.y, dir = blockIdx.z;
    const int ns = a.P - 1;
    const int c0 = g * q, c1 = min(c0 + q, ns) - 1;
    if (dir == 0 && g == 0) return;
    if (dir == 1 && g == G - 1) return;
    const double2 one = cmk<double2>(1.0, 0.0), mone = cmk<double2>(-1.0, 0.0);
    auto sep = [&](int c) { return c * a.m + a.m - 1; };
    auto out = [&](int c) { return Fs + (((size_t)s * ns + c) * 2 + dir) * BLK; };
    auto out32 = [&](int c) { return Fs32 ? Fs32 + (((size_t)s * ns + c) * 2 + dir) * BLK : nullptr; };
    const int first = dir == 0 ? c0 : c1;
    const int step = dir == 0 ? 1 : -1;
    const int sl = dir == 0 ? 1 : 2;                 // K_c in slot 1, U'_c in slot 2
    load_blk(Am, slot(a, s, sep(first), sl));
    __syncthreads();
    for (int idx = threadIdx.x; idx < WP * LDM; idx += NT) Am[idx] = cmul(Am[idx], mone);
    __syncthreads();
    store_blk(out(first), out32(first), Am, one);
    double2* cur = Am;
    double2* nxt = Bm;
    for (int c = first + step; c >= c0 && c <= c1; c += step) {
        gemm64_mfma(nxt, LDM, slot(a, s, sep(c), sl), WP, cur, LDM, mone, nullptr, 0);
        store_blk(out(c), out32(c), nxt, one);
        __syncthreads();
        double2* tmp = cur; cur = nxt; nxt = tmp;
    }
}

// Fc[((s*Ny + l)*2 + side)*8*WP + t*WP + k] = (side ? Y~ : X~)_l(tcol[s*8+t], k), interior rows
template <typename V>
__global__ void k_extract_targets(const V* __restrict__ F, V* __restrict__ Fc,
                                  const int* __restrict__ tcol, int Ny, int m, int P) {
    const int l = blockIdx.x, s = blockIdx.y;
    const int c = l / m;
    const bool sep = (c < P - 1) && (l == c * m + m - 1);
    for (int idx = threadIdx.x; idx < 2 * 8 * WP; idx += blockDim.x) {
        const int k = idx % WP, t = (idx / WP) % 8, side = idx / (8 * WP);
        const int q = tcol[s * 8 + t];
        V v; v.x = 0; v.y = 0;
        if (!sep && q >= 0) v = F[(((size_t)s * Ny + l) * NSLOT + 1 + side) * BLK + (size_t)k * WP + q];
        Fc[(((size_t)s * Ny + l) * 2 + side) * 8 * WP + t * WP + k] = v;
    }
}

FactorArgs make_args(const DevTables& t, const Geom& g, const Chunks& ch, double2* F, float2* F32, int* err) {
    FactorArgs a;
    a.F = F; a.F32 = F32; a.k2 = t.k2; a.ay = t.ay; a.ayh = t.ayh; a.cy = t.cy; a.by = t.by;
    a.sax = t.sax; a.saxh = t.saxh; a.scol = t.scol; a.sW = t.sW; a.err = err; a.rob = t.srob;
    a.Nx = g.Nx; a.Ny = g.Ny; a.m = ch.m; a.P = ch.P; a.inv_h2 = 1.0 / (g.h * g.h);
    return a;
}

}  // namespace

hipError_t launch_factor_chunks(const DevTables& t, const Geom& g, const Chunks& ch,
                                double2* F64, float2* F32, int* err, hipStream_t st) {
    FactorArgs a = make_args(t, g, ch, F64, F32, err);
    dim3 grid(ch.P, g.J);
    hipLaunchKernelGGL(k_factor_chunks, grid, dim3(NT), 0, st, a);
    hipLaunchKernelGGL(k_factor_spikes, dim3(ch.P, g.J, 2), dim3(NT), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_factor_separators(const DevTables& t, const Geom& g, const Chunks& ch,
                                    double2* F64, float2* F32, int* err, hipStream_t st) {
    if (ch.P < 2) return hipSuccess;
    FactorArgs a = make_args(t, g, ch, F64, F32, err);
    hipLaunchKernelGGL(k_factor_separators, dim3(g.J), dim3(NT), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_factor_propagators(const DevTables& t, const Geom& g, const Chunks& ch,
                                     const double2* F64, double2* Fs, float2* Fs32, hipStream_t st) {
    if (ch.G < 2) return hipSuccess;
    FactorArgs a = make_args(t, g, ch, const_cast<double2*>(F64), nullptr, nullptr);
    hipLaunchKernelGGL(k_factor_propagators, dim3(g.J, ch.G, 2), dim3(NT), 0, st, a, ch.q, ch.G, Fs, Fs32);
    return hipGetLastError();
}

template <typename V>
hipError_t launch_extract_targets(const V* F, V* Fc, const int* tcol, const Geom& g,
                                  const Chunks& ch, hipStream_t st) {
    hipLaunchKernelGGL((k_extract_targets<V>), dim3(g.Ny, g.J), dim3(256), 0, st, F, Fc, tcol,
                       g.Ny, ch.m, ch.P);
    return hipGetLastError();
}
template hipError_t launch_extract_targets<float2>(const float2*, float2*, const int*, const Geom&,
                                                   const Chunks&, hipStream_t);
template hipError_t launch_extract_targets<double2>(const double2*, double2*, const int*,
                                                    const Geom&, const Chunks&, hipStream_t);

}  // namespace helm

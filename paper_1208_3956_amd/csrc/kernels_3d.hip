// Slab factorisation and slab solves of the 3-D problem (Sec. 2.2 with the 7-point
// stencil; subdomains are slabs along x, Sec. 3 of the paper treats the 3-D case).
//
// A padded slab of W x-columns is block tridiagonal along y: block l holds the W * N_z
// unknowns (x, z) of the plane y = l, element k = z * W + x.  Its diagonal block T_l is
// the x- and z-part of the stencil plus the y-diagonal and -k^2; the couplings to the
// planes l -/+ 1 are the scalars c_l, b_l (the y-PML depends on y only).  Block LU along
// y (Algorithm 1 with blocks for rows):
//     S_0 = T_0,  S_l = T_l - c_l b_{l-1} S_{l-1}^{-1},  G_l = S_l^{-1}
//     forward   y_l = G_l (r_l - c_l y_{l-1})
//     backward  x_l = y_l - b_l G_l x_{l+1}
// The blocks are dense (B = W N_z up to ~2000), so the explicit inverses are computed in
// FP64 by blocked Gauss-Jordan elimination with partial pivoting over the whole column:
// per panel of NB columns one workgroup per slab reduces the panel (pivot search, row
// swap, scaling, elimination of every other row), then the remaining columns receive the
// panel's row swaps and one rank-NB update  A(:, J) += (C - E_K) A(K, J)  (a GEMM), where
// C holds the reduced panel columns.  The column exchanges that undo the pivoting are
// applied when the inverse is stored.  Every slab of one plane l is processed in the same
// launches (blockIdx.y / gridDim = slab); blocks are padded to Bp (a multiple of 64) with
// the identity.
//
// A solve step is one dense product per plane: G_l (Bp x Bp, column-major) times a panel
// of right-hand sides, each workgroup a 16-row x 16-column tile, with the right-hand side
// of the step (input field, transmission planes, previous plane) formed while it is
// staged.
#include "helm_internal.hpp"

namespace helm {

namespace {

constexpr int NB = 32;        // Gauss-Jordan panel width
constexpr int NTP = 512;      // threads of the panel kernel

__device__ inline double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// S = T_l - c_l b_{l-1} G_{l-1}  on every slab, identity on the padding
__global__ void __launch_bounds__(256) k3_build_S(Fac3Args a, int l, const double2* __restrict__ Gprev,
                                                  double2* __restrict__ S) {
    const int s = blockIdx.y;
    const size_t BB = (size_t)a.Bp * a.Bp;
    const int W = a.sW[s], B = W * a.Nz;
    double2 cb = make_double2(0.0, 0.0);
    if (l > 0) cb = cmul(a.cy[l], a.by[l - 1]);
    const double2 ay = a.ay[l], ayp = a.ayh[l + 1], aym = a.ayh[l];
    const double2 ydiag = cmul(ay, cadd(ayp, aym));
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < BB; e += (size_t)gridDim.x * blockDim.x) {
        const int col = (int)(e / a.Bp), row = (int)(e % a.Bp);
        double2 v = make_double2(0.0, 0.0);
        if (row < B && col < B) {
            if (l > 0) {
                const double2 gp = Gprev[(size_t)s * BB + e];
                v = cmk<double2>(-(cb.x * gp.x - cb.y * gp.y), -(cb.x * gp.y + cb.y * gp.x));
            }
            const int xr = row % W, zr = row / W, xc = col % W, zc = col / W;
            const double2* sax = a.sax + (size_t)s * WP;
            const double2* saxh = a.saxh + (size_t)s * (WP + 1);
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
        S[(size_t)s * BB + e] = v;
    }
}

// Gauss-Jordan on the panel columns [k0, k0 + NB) of every slab's matrix (one workgroup
// per slab): for each column k, the pivot is the largest |A(i, k)|, i >= k (the first of
// equal values), rows k and p are exchanged inside the panel, row k is divided by the
// pivot (A(k, k) becomes 1 / pivot) and every other row i loses A(i, k) times row k
// (A(i, k) becomes -A(i, k) / pivot).  perm[k] = p records the exchange.
__global__ void __launch_bounds__(NTP) k3_gj_panel(double2* __restrict__ S, int Bp, int k0,
                                                  int* __restrict__ perm, int* __restrict__ err) {
    const int s = blockIdx.x, t = threadIdx.x;
    double2* A = S + (size_t)s * Bp * Bp;
    __shared__ double2 rowk[NB];
    __shared__ double bv[NTP];
    __shared__ int bi[NTP];
    for (int k = k0; k < k0 + NB; ++k) {
        double best = -1.0;
        int arg = k;
        for (int i = k + t; i < Bp; i += NTP) {
            const double2 v = A[(size_t)k * Bp + i];
            const double m = v.x * v.x + v.y * v.y;
            if (m > best) { best = m; arg = i; }
        }
        bv[t] = best;
        bi[t] = arg;
        __syncthreads();
        for (int w = NTP / 2; w > 0; w >>= 1) {
            if (t < w) {
                const double o = bv[t + w];
                const int oi = bi[t + w];
                if (o > bv[t] || (o == bv[t] && oi < bi[t])) { bv[t] = o; bi[t] = oi; }
            }
            __syncthreads();
        }
        int p = bi[0];
        const bool bad = !(bv[0] > 0.0) || !isfinite(bv[0]);
        __syncthreads();
        if (bad) {
            p = k;
            if (t == 0) err[0] = 1;
        }
        if (t == 0) perm[(size_t)s * Bp + k] = p;
        if (p != k) {
            for (int c = t; c < NB; c += NTP) {
                double2* col = A + (size_t)(k0 + c) * Bp;
                const double2 x = col[k];
                col[k] = col[p];
                col[p] = x;
            }
        }
        __syncthreads();
        double2 piv = A[(size_t)k * Bp + k];
        if (bad) piv = make_double2(1.0, 0.0);
        __syncthreads();                 // every thread holds the pivot before row k changes
        for (int c = t; c < NB; c += NTP) {
            const int cc = k0 + c;
            const double2 v = cc == k ? make_double2(1.0, 0.0) : A[(size_t)cc * Bp + k];
            const double2 q = cdiv(v, piv);
            rowk[c] = q;
            A[(size_t)cc * Bp + k] = q;
        }
        __syncthreads();
        for (int i = t; i < Bp; i += NTP) {
            if (i == k) continue;
            const double2 m = A[(size_t)k * Bp + i];
            if (m.x == 0.0 && m.y == 0.0) continue;
#pragma unroll 4
            for (int c = 0; c < NB; ++c) {
                const int cc = k0 + c;
                double2* p2 = A + (size_t)cc * Bp + i;
                const double2 old = cc == k ? make_double2(0.0, 0.0) : *p2;
                *p2 = csub(old, cmul(m, rowk[c]));
            }
        }
        __syncthreads();
    }
}

// Outside the panel: the panel's row exchanges (in order) and the operands of the update,
// Tm(kk, j) = A(k0 + kk, j) for j outside the panel (0 inside),  Cm(i, kk) = C(i, kk) - [i = k0 + kk].
__global__ void __launch_bounds__(256) k3_gj_prep(double2* __restrict__ S, int Bp, int k0,
                                                 const int* __restrict__ perm, double2* __restrict__ Tm,
                                                 double2* __restrict__ Cm) {
    const int s = blockIdx.y;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= Bp) return;
    double2* A = S + (size_t)s * Bp * Bp;
    const int* pm = perm + (size_t)s * Bp;
    const bool inK = j >= k0 && j < k0 + NB;
    double2* col = A + (size_t)j * Bp;
    double2* tm = Tm + ((size_t)s * Bp + j) * NB;
    if (!inK) {
        for (int k = k0; k < k0 + NB; ++k) {
            const int p = pm[k];
            if (p != k) {
                const double2 x = col[k];
                col[k] = col[p];
                col[p] = x;
            }
        }
        for (int kk = 0; kk < NB; ++kk) tm[kk] = col[k0 + kk];
    } else {
        for (int kk = 0; kk < NB; ++kk) tm[kk] = make_double2(0.0, 0.0);
    }
    // row j of the panel columns
    double2* cm = Cm + (size_t)s * Bp * NB;
    for (int kk = 0; kk < NB; ++kk) {
        double2 v = A[(size_t)(k0 + kk) * Bp + j];
        if (j == k0 + kk) v.x -= 1.0;
        cm[(size_t)kk * Bp + j] = v;
    }
}

// A(:, :) += Cm Tm  (Bp x NB times NB x Bp), 64 x 64 tiles, thread = 4 x 4 outputs
__global__ void __launch_bounds__(256) k3_gemm_update(double2* __restrict__ S, int Bp,
                                                     const double2* __restrict__ Tm,
                                                     const double2* __restrict__ Cm) {
    const int s = blockIdx.z;
    const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
    const int t = threadIdx.x, ty = t / 16, tx = t % 16;
    __shared__ double2 Cs[NB][64];
    __shared__ double2 Ts[NB][64];
    const double2* cm = Cm + (size_t)s * Bp * NB;
    const double2* tm = Tm + (size_t)s * Bp * NB;
    for (int e = t; e < NB * 64; e += 256) {
        const int kk = e / 64, ii = e % 64;
        Cs[kk][ii] = cm[(size_t)kk * Bp + i0 + ii];
        const int jj = e / NB, k2 = e % NB;
        Ts[k2][jj] = tm[(size_t)(j0 + jj) * NB + k2];
    }
    __syncthreads();
    double2 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0.0, 0.0);
    for (int kk = 0; kk < NB; ++kk) {
        double2 cv[4], tv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) cv[a] = Cs[kk][tx + 16 * a];
#pragma unroll
        for (int b = 0; b < 4; ++b) tv[b] = Ts[kk][ty + 16 * b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) cfma(acc[a][b], cv[a], tv[b]);
    }
    double2* A = S + (size_t)s * Bp * Bp;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        double2* col = A + (size_t)(j0 + ty + 16 * b) * Bp + i0;
#pragma unroll
        for (int a = 0; a < 4; ++a) col[tx + 16 * a] = cadd(col[tx + 16 * a], acc[a][b]);
    }
}

// Column exchanges that finish the inverse, as one permutation: applying the exchanges
// k <-> perm[k] in order k = 0, 1, ... to the values, who[x] ends as the column index
// that lands on x; the inverse's column j is column pi[j] of the reduced matrix.
__global__ void __launch_bounds__(256) k3_gj_perm(const int* __restrict__ perm, int Bp,
                                                 int* __restrict__ pi) {
    const int s = blockIdx.x;
    const int* pm = perm + (size_t)s * Bp;
    __shared__ int wh[BP3_MAX];
    for (int x = threadIdx.x; x < Bp; x += 256) wh[x] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < Bp; ++k) {
            const int p = pm[k];
            if (p != k) { const int a = wh[k]; wh[k] = wh[p]; wh[p] = a; }
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < Bp; x += 256) pi[(size_t)s * Bp + wh[x]] = x;
}

// G(:, j) = A(:, pi[j]) into the FP64 copy used by the next plane (if any) and the stored
// factor in the working precision T
template <typename T>
__global__ void __launch_bounds__(256) k3_store(const double2* __restrict__ S, int Bp, const int* __restrict__ pi,
                                               double2* __restrict__ G64, cplx<T>* __restrict__ out,
                                               size_t out_stride) {
    const int s = blockIdx.y, j = blockIdx.x;
    const size_t BB = (size_t)Bp * Bp;
    const double2* src = S + s * BB + (size_t)pi[(size_t)s * Bp + j] * Bp;
    for (int i = threadIdx.x; i < Bp; i += 256) {
        const double2 v = src[i];
        if (G64) G64[s * BB + (size_t)j * Bp + i] = v;
        out[s * out_stride + (size_t)j * Bp + i] = ccast<cplx<T>>(v);
    }
}

// ---------------------------------------------------------------- slab solve steps
template <typename T>
__device__ inline cplx<T> gather3(const Solve3Args<T>& a, int r, int l, int k) {
    const IOSpec& io = a.io;
    const int q = k % a.W, z = k / a.W;
    const size_t rho = (size_t)z * a.Ny + l;
    double2 v = make_double2(0.0, 0.0);
    if (q >= io.src_lo && q < io.src_hi)
        v = io.src[(size_t)r * io.src_rs + rho * io.src_ls + (q + io.src_off)];
    if (io.q_t >= 0 && (q == io.q_t || q == io.q_t + 1)) {
        const double2 ta = io.trA[(size_t)r * a.Nrow + rho], tb = io.trB[(size_t)r * a.Nrow + rho];
        v.x += io.coef * (tb.x - ta.x);
        v.y += io.coef * (tb.y - ta.y);
    }
    return ccast<cplx<T>>(v);
}

template <typename T>
__device__ inline void scatter3(const Solve3Args<T>& a, int r, int l, int k, cplx<T> x) {
    const IOSpec& io = a.io;
    const int q = k % a.W, z = k / a.W;
    const size_t rho = (size_t)z * a.Ny + l;
    const double2 xv = ccast<double2>(x);
    const bool o = (q >= io.o_lo[0] && q < io.o_hi[0]) || (q >= io.o_lo[1] && q < io.o_hi[1]);
    if (o && io.dst) {
        double2* p = io.dst + (size_t)r * io.dst_rs + rho * io.dst_ls + (q + io.dst_off);
        *p = io.accumulate ? cadd(*p, xv) : xv;
    }
    if (q == io.qo0 && io.tro0) io.tro0[(size_t)r * a.Nrow + rho] = xv;
    if (q == io.qo1 && io.tro1) io.tro1[(size_t)r * a.Nrow + rho] = xv;
}

// One plane of the forward (FWD) or backward substitution for 16 rows x 16 right-hand
// sides per workgroup:  FWD  y_l = G_l (r_l - c_l y_{l-1});  BWD  x_l = y_l - G_l (b_l x_{l+1}).
// Yw holds y (then x) as [l][k][RP].
template <typename T, bool FWD>
__global__ void __launch_bounds__(256) k3_step(Solve3Args<T> a, int l) {
    using V = cplx<T>;
    constexpr int KC = 64;
    __shared__ V Gs[KC][16];
    __shared__ V Ts[KC][16];
    const int t = threadIdx.x, ti = t % 16, tj = t / 16;
    const int i0 = blockIdx.x * 16, r0 = blockIdx.y * 16;
    const V* G = a.F + (size_t)l * a.Bp * a.Bp;
    const size_t plane = (size_t)a.Bp * a.RP;
    V coupling;
    const V* vin;
    if (FWD) {
        const double2 c = a.cy[l];
        coupling = cmk<V>((decltype(V{}.x))c.x, (decltype(V{}.x))c.y);
        vin = l > 0 ? a.Yw + (size_t)(l - 1) * plane : nullptr;
    } else {
        const double2 b = a.by[l];
        coupling = cmk<V>((decltype(V{}.x))b.x, (decltype(V{}.x))b.y);
        vin = a.Yw + (size_t)(l + 1) * plane;
    }
    V acc = cmk<V>(0, 0);
    for (int k0 = 0; k0 < a.B; k0 += KC) {
        for (int e = t; e < KC * 16; e += 256) {
            const int kk = e / 16, ii = e % 16, k = k0 + kk;
            Gs[kk][ii] = k < a.B ? G[(size_t)k * a.Bp + i0 + ii] : cmk<V>(0, 0);
            const int r = r0 + ii;   // e % 16 indexes the right-hand side here
            V tv = cmk<V>(0, 0);
            if (k < a.B && r < a.nrhs) {
                if (FWD) {
                    tv = gather3<T>(a, r, l, k);
                    if (vin) tv = csub(tv, cmul(coupling, vin[(size_t)k * a.RP + r]));
                } else {
                    tv = cmul(coupling, vin[(size_t)k * a.RP + r]);
                }
            }
            Ts[kk][ii] = tv;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < KC; ++kk) cfma(acc, Gs[kk][ti], Ts[kk][tj]);
        __syncthreads();
    }
    const int i = i0 + ti, r = r0 + tj;
    if (i >= a.B || r >= a.nrhs) return;
    V* yl = a.Yw + (size_t)l * plane + (size_t)i * a.RP + r;
    if (FWD) {
        *yl = acc;
        if (l == a.Ny - 1) scatter3<T>(a, r, l, i, acc);
    } else {
        const V x = csub(*yl, acc);
        *yl = x;
        scatter3<T>(a, r, l, i, x);
    }
}

}  // namespace

hipError_t launch_factor3_plane(const Fac3Args& a, int l, const double2* Gprev, double2* S,
                                double2* Tm, double2* Cm, int* perm, int* pi, int* err,
                                double2* G64, void* out, bool out_single, size_t out_stride,
                                hipStream_t st) {
    const size_t BB = (size_t)a.Bp * a.Bp;
    unsigned nb = (unsigned)std::min<size_t>((BB + 255) / 256, 4096);
    hipLaunchKernelGGL(k3_build_S, dim3(nb, a.J), dim3(256), 0, st, a, l, Gprev, S);
    for (int k0 = 0; k0 < a.Bp; k0 += NB) {
        hipLaunchKernelGGL(k3_gj_panel, dim3(a.J), dim3(NTP), 0, st, S, a.Bp, k0, perm, err);
        hipLaunchKernelGGL(k3_gj_prep, dim3((a.Bp + 255) / 256, a.J), dim3(256), 0, st, S, a.Bp, k0, perm, Tm, Cm);
        hipLaunchKernelGGL(k3_gemm_update, dim3(a.Bp / 64, a.Bp / 64, a.J), dim3(256), 0, st, S, a.Bp, Tm, Cm);
    }
    hipLaunchKernelGGL(k3_gj_perm, dim3(a.J), dim3(256), 0, st, perm, a.Bp, pi);
    if (out_single)
        hipLaunchKernelGGL(k3_store<float>, dim3(a.Bp, a.J), dim3(256), 0, st, S, a.Bp, pi, G64,
                           static_cast<float2*>(out), out_stride);
    else
        hipLaunchKernelGGL(k3_store<double>, dim3(a.Bp, a.J), dim3(256), 0, st, S, a.Bp, pi, G64,
                           static_cast<double2*>(out), out_stride);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_strip_solve3(const Solve3Args<T>& a, hipStream_t st, KTimer* kt) {
    dim3 grid(a.Bp / 16, a.RP / 16);
    if (kt) kt->begin(K_PHASE_A, st);
    for (int l = 0; l < a.Ny; ++l) hipLaunchKernelGGL((k3_step<T, true>), grid, dim3(256), 0, st, a, l);
    for (int l = a.Ny - 2; l >= 0; --l) hipLaunchKernelGGL((k3_step<T, false>), grid, dim3(256), 0, st, a, l);
    if (kt) kt->end(K_PHASE_A, st);
    return hipGetLastError();
}

template hipError_t launch_strip_solve3<float>(const Solve3Args<float>&, hipStream_t, KTimer*);
template hipError_t launch_strip_solve3<double>(const Solve3Args<double>&, hipStream_t, KTimer*);

}  // namespace helm

namespace helm {
size_t factor3_panel_width() { return NB; }
}  // namespace helm

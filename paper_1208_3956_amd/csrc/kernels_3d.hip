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
// A solve step is one dense product per plane: G_l (Bp x Bp) times a panel of right-hand
// sides ([k][RP], right-hand sides fastest; complex64 in pairs of k), each workgroup a
// 16-row x 16-column tile with its waves splitting the k range.  Operands are read straight
// from global memory in the MFMA lane layout.  The right-hand side of the next forward
// plane (input field, transmission planes, minus c_{l+1} y_l) is formed by the tile that
// computes y_l, so every element is gathered once.
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

// The same reduction of the panel [k0, k0 + NB) with the panel itself blocked: inner panels
// of NI columns are reduced in LDS (pivot search, exchange, scaling, elimination of all other
// rows), written back, and applied to the other columns of the panel as one rank-NI update
// (after their row exchanges).  The panel's global traffic drops from NB passes over NB
// columns to about NB / NI passes.  Requires Bp <= BPI_MAX (the inner panel lives in LDS).
constexpr int NI = 4;
constexpr int BPI_MAX = 2048;
constexpr int NTI = 1024;

__global__ void __launch_bounds__(NTI) k3_gj_panel_lds(double2* __restrict__ S, int Bp, int k0,
                                                      int* __restrict__ perm, int* __restrict__ err) {
    const int s = blockIdx.x, t = threadIdx.x;
    double2* A = S + (size_t)s * Bp * Bp;
    __shared__ double2 Ps[NI][BPI_MAX];
    __shared__ double2 rowk[NI];
    __shared__ double2 tv[NB][NI];
    __shared__ double bv[NTI / 64];
    __shared__ int bi[NTI / 64];
    __shared__ int pv[NI];
    for (int ki = k0; ki < k0 + NB; ki += NI) {
        for (int e = t; e < NI * Bp; e += NTI) Ps[e / Bp][e % Bp] = A[(size_t)(ki + e / Bp) * Bp + e % Bp];
        __syncthreads();
        for (int kk = 0; kk < NI; ++kk) {
            const int k = ki + kk;
            // pivot: largest |P(i, kk)|, i >= k, first of equal values
            double best = -1.0;
            int arg = k;
            for (int i = k + t; i < Bp; i += NTI) {
                const double2 v = Ps[kk][i];
                const double m = v.x * v.x + v.y * v.y;
                if (m > best) { best = m; arg = i; }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ob = __shfl_xor(best, off);
                const int oa = __shfl_xor(arg, off);
                if (ob > best || (ob == best && oa < arg)) { best = ob; arg = oa; }
            }
            if ((t & 63) == 0) { bv[t >> 6] = best; bi[t >> 6] = arg; }
            __syncthreads();
            if (t == 0) {
                double b = bv[0];
                int a = bi[0];
                for (int w = 1; w < NTI / 64; ++w)
                    if (bv[w] > b || (bv[w] == b && bi[w] < a)) { b = bv[w]; a = bi[w]; }
                const bool bad = !(b > 0.0) || !isfinite(b);
                if (bad) { a = k; err[0] = 1; }
                pv[kk] = a;
                perm[(size_t)s * Bp + k] = a;
            }
            __syncthreads();
            const int p = pv[kk];
            if (p != k && t < NI) {
                const double2 x = Ps[t][k];
                Ps[t][k] = Ps[t][p];
                Ps[t][p] = x;
            }
            __syncthreads();
            if (t < NI) {
                double2 piv = Ps[kk][k];
                if (!(piv.x * piv.x + piv.y * piv.y > 0.0)) piv = make_double2(1.0, 0.0);
                const double2 v = t == kk ? make_double2(1.0, 0.0) : Ps[t][k];
                rowk[t] = cdiv(v, piv);
            }
            __syncthreads();
            for (int i = t; i < Bp; i += NTI) {
                if (i == k) {
#pragma unroll
                    for (int c = 0; c < NI; ++c) Ps[c][i] = rowk[c];
                } else {
                    const double2 m = Ps[kk][i];
#pragma unroll
                    for (int c = 0; c < NI; ++c) {
                        const double2 old = c == kk ? make_double2(0.0, 0.0) : Ps[c][i];
                        Ps[c][i] = csub(old, cmul(m, rowk[c]));
                    }
                }
            }
            __syncthreads();
        }
        // the reduced inner columns back to global memory
        for (int e = t; e < NI * Bp; e += NTI) A[(size_t)(ki + e / Bp) * Bp + e % Bp] = Ps[e / Bp][e % Bp];
        // the other columns of the panel: the inner exchanges, then the rank-NI update
        // A(:, j) += (C - E) A(K_in, j)
        if (t < NB) {
            const int j = k0 + t;
            if (j < ki || j >= ki + NI) {
                double2* col = A + (size_t)j * Bp;
                for (int kk = 0; kk < NI; ++kk) {
                    const int k = ki + kk, p = pv[kk];
                    if (p != k) { const double2 x = col[k]; col[k] = col[p]; col[p] = x; }
                }
#pragma unroll
                for (int kk = 0; kk < NI; ++kk) tv[t][kk] = col[ki + kk];
            }
        }
        __syncthreads();
        for (int e = t; e < NB * Bp; e += NTI) {
            const int jj = e / Bp, i = e % Bp, j = k0 + jj;
            if (j >= ki && j < ki + NI) continue;
            double2 acc = make_double2(0.0, 0.0);
#pragma unroll
            for (int kk = 0; kk < NI; ++kk) {
                double2 c = Ps[kk][i];
                if (i == ki + kk) c.x -= 1.0;
                acc = cadd(acc, cmul(c, tv[jj][kk]));
            }
            double2* q = A + (size_t)j * Bp + i;
            *q = cadd(*q, acc);
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
// Plane vectors [k][RP]: complex128 stores entry (k, r) at k RP + r; complex64 in pairs of
// k, at 2 ((k / 2) RP + r) + k % 2, so that a lane's two k of a pair come in one 16-byte load
// and the 16 lanes of a right-hand-side tile read 256 contiguous bytes.
template <typename T>
__device__ inline size_t pidx(int k, int r, int RP) { return (size_t)k * RP + r; }
template <>
__device__ inline size_t pidx<float>(int k, int r, int RP) { return 2 * ((size_t)(k >> 1) * RP + r) + (k & 1); }

template <typename T>
__device__ inline cplx<T> gather3(const Solve3Args<T>& a, int r, int l, int k) {
    const IOSpec& io = a.io;
    const int q = k % a.W, z = k / a.W;
    const size_t rho = (size_t)z * a.Ny + l;
    double2 v = make_double2(0.0, 0.0);
    if (q >= io.src_lo && q < io.src_hi)
        v = io.src[(size_t)r * io.src_rs + rho * io.src_ls + (q + io.src_off)];
    if (tr_col(io, q)) {
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
    const bool o0 = q >= io.o_lo[0] && q < io.o_hi[0];
    const bool o = o0 || (q >= io.o_lo[1] && q < io.o_hi[1]);
    if (o && io.dst) {
        double2* p = io.dst + (size_t)r * io.dst_rs + rho * io.dst_ls + (q + io.dst_off[o0 ? 0 : 1]);
        *p = io.accumulate ? cadd(*p, xv) : xv;
    }
    if (q == io.qo0 && io.tro0) io.tro0[(size_t)r * a.Nrow + rho] = xv;
    if (q == io.qo1 && io.tro1) io.tro1[(size_t)r * a.Nrow + rho] = xv;
}

typedef float mf4 __attribute__((ext_vector_type(4)));

// Right-hand side of plane 0: Tw[i][r] = r_0(i, r), zero on the padding rows and on the
// right-hand-side columns beyond nrhs.
template <typename T>
__global__ void __launch_bounds__(256) k3_rhs0(Solve3Args<T> a, cplx<T>* __restrict__ Tw) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)a.Bp * a.RP) return;
    const int i = (int)(e / a.RP), r = (int)(e % a.RP);
    Tw[pidx<T>(i, r, a.RP)] = (i < a.B && r < a.nrhs) ? gather3<T>(a, r, 0, i) : cmk<cplx<T>>(0, 0);
}

// Z = G X for a 16-row x 16-column tile: G Bp x Bp, column-major (complex128) or in 16-row
// panels (complex64: entry (i, k) at (i / 16) 16 Bp + 32 (k / 2) + 2 (i % 16) + k % 2, so
// that the 16 rows of a tile are one contiguous run of 16 Bp entries and each row's pairs of
// k are adjacent), X a plane vector (pidx).  The k range
// is cut into blocks of 16; wave w of NW3 takes blocks w, w + NW3, ... (several waves per
// SIMD hide the load latency; each wave also loads its next block before it multiplies
// the current one).  The NW3 partial tiles are added through LDS.  Returns, for thread
// t < 256, the entry (row t / 16, column t % 16) of the tile.
// complex64: v_mfma_f32_16x16x4f32, three real products per complex one (Gauss's form;
// lane layout A[l % 16][l / 16], B[l / 16][l % 16], C[4 (l / 16) + j][l % 16] in
// component j).
constexpr int NW3 = 16;
constexpr int NT3 = 64 * NW3;

__device__ inline float2 tile_product(const float2* __restrict__ G, const float2* __restrict__ X, int Bp,
                                      int RP, int i0, int r0, float2 (*red)[16][16]) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, n = lane & 15, q4 = lane >> 4;
    const int nblk = Bp / 16;
    // complex products from three real ones: x1 = sum Gr Xr, x2 = sum Gi Xi,
    // x3 = sum (Gr + Gi)(Xr + Xi); Re = x1 - x2, Im = x3 - x1 - x2 (two chains of each for
    // independent MFMAs)
    mf4 x1a = {0.f, 0.f, 0.f, 0.f}, x2a = x1a, x3a = x1a, x1b = x1a, x2b = x1a, x3b = x1a;
    // k-step u of block b: lane (n, q4) takes k = 16 b + 4 q4 + u (a permutation of the
    // block's k, the same for both operands); k-steps 2p, 2p + 1 are one pair of both layouts
    const float2* gp = G + (size_t)(i0 / 16) * 16 * Bp + 64 * q4 + 2 * n;
    const float2* xp = X + 2 * ((size_t)(2 * q4) * RP + r0 + n);
    float2 g[4], x[4], gn[4], xn[4];
    auto load = [&](int b, float2 (&gg)[4], float2 (&xx)[4]) {
        const float4* G4 = reinterpret_cast<const float4*>(gp + 256 * (size_t)b);
        const float4* X4 = reinterpret_cast<const float4*>(xp + 16 * (size_t)b * RP);
        const float4 g01 = G4[0], g23 = G4[16], x01 = X4[0], x23 = X4[RP];
        gg[0] = make_float2(g01.x, g01.y); gg[1] = make_float2(g01.z, g01.w);
        gg[2] = make_float2(g23.x, g23.y); gg[3] = make_float2(g23.z, g23.w);
        xx[0] = make_float2(x01.x, x01.y); xx[1] = make_float2(x01.z, x01.w);
        xx[2] = make_float2(x23.x, x23.y); xx[3] = make_float2(x23.z, x23.w);
    };
    if (w < nblk) load(w, g, x);
    for (int b = w; b < nblk; b += NW3) {
        const int bn = b + NW3 < nblk ? b + NW3 : b;     // clamped: the last prefetch is a re-read
        load(bn, gn, xn);
#pragma unroll
        for (int u = 0; u < 4; u += 2) {
            x1a = __builtin_amdgcn_mfma_f32_16x16x4f32(g[u].x, x[u].x, x1a, 0, 0, 0);
            x2a = __builtin_amdgcn_mfma_f32_16x16x4f32(g[u].y, x[u].y, x2a, 0, 0, 0);
            x3a = __builtin_amdgcn_mfma_f32_16x16x4f32(g[u].x + g[u].y, x[u].x + x[u].y, x3a, 0, 0, 0);
            x1b = __builtin_amdgcn_mfma_f32_16x16x4f32(g[u + 1].x, x[u + 1].x, x1b, 0, 0, 0);
            x2b = __builtin_amdgcn_mfma_f32_16x16x4f32(g[u + 1].y, x[u + 1].y, x2b, 0, 0, 0);
            x3b = __builtin_amdgcn_mfma_f32_16x16x4f32(g[u + 1].x + g[u + 1].y, x[u + 1].x + x[u + 1].y, x3b, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) { g[u] = gn[u]; x[u] = xn[u]; }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float p1 = x1a[j] + x1b[j], p2 = x2a[j] + x2b[j], p3 = x3a[j] + x3b[j];
        red[w][4 * q4 + j][n] = make_float2(p1 - p2, p3 - p1 - p2);
    }
    __syncthreads();
    float2 z = make_float2(0.f, 0.f);
    if (t < 256) {
        const int i = t >> 4, c = t & 15;
#pragma unroll
        for (int v = 0; v < NW3; ++v) { z.x += red[v][i][c].x; z.y += red[v][i][c].y; }
    }
    return z;
}

// complex128: FMA, each lane four rows (4 (l / 16) + j) of one column (l % 16)
__device__ inline double2 tile_product(const double2* __restrict__ G, const double2* __restrict__ X, int Bp,
                                       int RP, int i0, int r0, double2 (*red)[16][16]) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, n = lane & 15, q4 = lane >> 4;
    const int nblk = Bp / 16;
    double2 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = make_double2(0.0, 0.0);
    const double2* gp = G + i0 + 4 * q4;
    const double2* xp = X + r0 + n;
    for (int b = w; b < nblk; b += NW3) {
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
            const int k = 16 * b + kk;
            const double2 xv = xp[(size_t)k * RP];
#pragma unroll
            for (int j = 0; j < 4; ++j) cfma(acc[j], gp[(size_t)k * Bp + j], xv);
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) red[w][4 * q4 + j][n] = acc[j];
    __syncthreads();
    double2 z = make_double2(0.0, 0.0);
    if (t < 256) {
        const int i = t >> 4, c = t & 15;
#pragma unroll
        for (int v = 0; v < NW3; ++v) { z.x += red[v][i][c].x; z.y += red[v][i][c].y; }
    }
    return z;
}

// Forward plane l: y_l = G_l Tw_l, kept in Yw[l]; the tile's rows of the next right-hand
// side Tn = r_{l+1} - c_{l+1} y_l are formed here (the last plane scatters x = y instead).
template <typename T>
__global__ void __launch_bounds__(NT3) k3_fwd(Solve3Args<T> a, int l, const cplx<T>* __restrict__ Tw,
                                             cplx<T>* __restrict__ Tn) {
    using V = cplx<T>;
    __shared__ V red[NW3][16][16];
    const int i0 = blockIdx.x * 16, r0 = blockIdx.y * 16;
    const V y = tile_product(a.F + (size_t)l * a.Bp * a.Bp, Tw, a.Bp, a.RP, i0, r0, red);
    if (threadIdx.x >= 256) return;
    const int i = i0 + (threadIdx.x >> 4), r = r0 + (threadIdx.x & 15);
    const size_t at = pidx<T>(i, r, a.RP);
    a.Yw[(size_t)l * a.Bp * a.RP + at] = y;
    const bool live = i < a.B && r < a.nrhs;
    if (l + 1 < a.Ny) {
        V tn = cmk<V>(0, 0);
        if (live) {
            const double2 c = a.cy[l + 1];
            tn = csub(gather3<T>(a, r, l + 1, i), cmul(ccast<V>(c), y));
        }
        Tn[at] = tn;
    } else if (live) {
        scatter3<T>(a, r, l, i, y);
    }
}

// Backward plane l: x_l = y_l - b_l G_l x_{l+1}, kept in Yw[l] and scattered.
template <typename T>
__global__ void __launch_bounds__(NT3) k3_bwd(Solve3Args<T> a, int l) {
    using V = cplx<T>;
    __shared__ V red[NW3][16][16];
    const int i0 = blockIdx.x * 16, r0 = blockIdx.y * 16;
    const size_t plane = (size_t)a.Bp * a.RP;
    const V z = tile_product(a.F + (size_t)l * a.Bp * a.Bp, a.Yw + (size_t)(l + 1) * plane, a.Bp, a.RP,
                             i0, r0, red);
    if (threadIdx.x >= 256) return;
    const int i = i0 + (threadIdx.x >> 4), r = r0 + (threadIdx.x & 15);
    V* yl = a.Yw + (size_t)l * plane + pidx<T>(i, r, a.RP);
    const V x = csub(*yl, cmul(ccast<V>(a.by[l]), z));
    *yl = x;
    if (i < a.B && r < a.nrhs) scatter3<T>(a, r, l, i, x);
}

// The complex64 inverses of plane l of the J slots (column-major, slot stride `stride`)
// written to dst[s][Bp^2] in the 16-row panel layout of the sweeps (destination order:
// panel, pair of columns, row within the panel, column within the pair; the reads are
// 16-entry runs of two columns).
__global__ void __launch_bounds__(256) k3_panelize(const float2* __restrict__ F, size_t stride, int l, int Bp,
                                                  float2* __restrict__ dst) {
    const size_t BB = (size_t)Bp * Bp, PW = (size_t)16 * Bp;
    const float2* src = F + blockIdx.y * stride + (size_t)l * BB;
    float2* d = dst + blockIdx.y * BB;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < BB; e += (size_t)gridDim.x * 256) {
        const size_t p = e / PW, rem = e % PW, k = 2 * (rem / 32) + rem % 2, ii = (rem % 32) / 2;
        d[e] = src[k * Bp + 16 * p + ii];
    }
}

// dst[s][Bp^2] back into plane l of slot s
__global__ void __launch_bounds__(256) k3_plane_back(float2* __restrict__ F, size_t stride, int l, int Bp,
                                                    const float2* __restrict__ src) {
    const size_t BB = (size_t)Bp * Bp;
    float2* d = F + blockIdx.y * stride + (size_t)l * BB;
    const float2* q = src + blockIdx.y * BB;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < BB; e += (size_t)gridDim.x * 256) d[e] = q[e];
}

}  // namespace

hipError_t launch_factor3_panelize(float2* F, size_t stride, int J, int Ny, int Bp, float2* work, hipStream_t st) {
    const size_t BB = (size_t)Bp * Bp;
    const unsigned nb = (unsigned)std::min<size_t>((BB + 255) / 256, 2048);
    for (int l = 0; l < Ny; ++l) {
        hipLaunchKernelGGL(k3_panelize, dim3(nb, J), dim3(256), 0, st, F, stride, l, Bp, work);
        hipLaunchKernelGGL(k3_plane_back, dim3(nb, J), dim3(256), 0, st, F, stride, l, Bp, work);
    }
    return hipGetLastError();
}

hipError_t launch_factor3_plane(const Fac3Args& a, int l, const double2* Gprev, double2* S,
                                double2* Tm, double2* Cm, int* perm, int* pi, int* err,
                                double2* G64, void* out, bool out_single, size_t out_stride,
                                hipStream_t st) {
    const size_t BB = (size_t)a.Bp * a.Bp;
    unsigned nb = (unsigned)std::min<size_t>((BB + 255) / 256, 4096);
    hipLaunchKernelGGL(k3_build_S, dim3(nb, a.J), dim3(256), 0, st, a, l, Gprev, S);
    for (int k0 = 0; k0 < a.Bp; k0 += NB) {
        if (a.Bp <= BPI_MAX)
            hipLaunchKernelGGL(k3_gj_panel_lds, dim3(a.J), dim3(NTI), 0, st, S, a.Bp, k0, perm, err);
        else
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
    cplx<T>* Tw[2] = {a.Tw, a.Tw + (size_t)a.Bp * a.RP};
    if (kt) kt->begin(K_PHASE_A, st);
    hipLaunchKernelGGL(k3_rhs0<T>, dim3((unsigned)(((size_t)a.Bp * a.RP + 255) / 256)), dim3(256), 0, st, a, Tw[0]);
    for (int l = 0; l < a.Ny; ++l)
        hipLaunchKernelGGL(k3_fwd<T>, grid, dim3(NT3), 0, st, a, l, Tw[l & 1], Tw[(l + 1) & 1]);
    for (int l = a.Ny - 2; l >= 0; --l) hipLaunchKernelGGL(k3_bwd<T>, grid, dim3(NT3), 0, st, a, l);
    if (kt) kt->end(K_PHASE_A, st);
    return hipGetLastError();
}

template hipError_t launch_strip_solve3<float>(const Solve3Args<float>&, hipStream_t, KTimer*);
template hipError_t launch_strip_solve3<double>(const Solve3Args<double>&, hipStream_t, KTimer*);

}  // namespace helm

namespace helm {
size_t factor3_panel_width() { return NB; }
}  // namespace helm

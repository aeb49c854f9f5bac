// FP64 kernels on whole fields: the PML stencil (Sec. 2.2) and the batched vector
// operations of right-preconditioned GMRES (Sec. 2.3).
//
// Fields are [nrhs][Ny][Nx] complex128 ([nrhs][Nz][Ny][Nx] in 3-D), x fastest.  Reductions are deterministic: every
// block reduces in a fixed tree and the per-block partial sums are added in block order.
#include "helm_internal.hpp"

namespace helm {

namespace {

struct StencilArgs {
    const double* k2;
    const double2* ax;
    const double2* axh;
    const double2* ay;
    const double2* ayh;
    const double2* az;     // 3-D only (null in 2-D)
    const double2* azh;
    int Nx, Ny, Nz;
    double inv_h2;
};

// (A u) at (l, i) in the paper form:
//   -alpha_x(i)/h^2 [alpha_x(i+1/2)(u_{i+1}-u_i) - alpha_x(i-1/2)(u_i-u_{i-1})]
//   -alpha_y(l)/h^2 [alpha_y(l+1/2)(u_{l+1}-u_l) - alpha_y(l-1/2)(u_l-u_{l-1})] - k^2 u
// with zero Dirichlet ghosts; in 3-D the same z-term is added (7-point stencil).  `row`
// is z * Ny + l.
__device__ inline double2 stencil_at(const StencilArgs& s, const double2* __restrict__ u, int row, int i) {
    const int l = row % s.Ny, z = row / s.Ny;
    const size_t p = (size_t)row * s.Nx + i;
    const double2 uc = u[p];
    const double2 ue = (i + 1 < s.Nx) ? u[p + 1] : cmk<double2>(0, 0);
    const double2 uw = (i > 0) ? u[p - 1] : cmk<double2>(0, 0);
    const double2 un = (l + 1 < s.Ny) ? u[p + s.Nx] : cmk<double2>(0, 0);
    const double2 us = (l > 0) ? u[p - s.Nx] : cmk<double2>(0, 0);
    const double2 ae = s.axh[i + 1], aw = s.axh[i];
    const double2 an = s.ayh[l + 1], as = s.ayh[l];
    // x part: alpha_x(i) [ae (uc - ue) + aw (uc - uw)]
    double2 xp = cadd(cmul(ae, csub(uc, ue)), cmul(aw, csub(uc, uw)));
    xp = cmul(s.ax[i], xp);
    double2 yp = cadd(cmul(an, csub(uc, un)), cmul(as, csub(uc, us)));
    yp = cmul(s.ay[l], yp);
    double2 r = cadd(xp, yp);
    if (s.Nz > 1) {
        const size_t pl = (size_t)s.Ny * s.Nx;
        const double2 uu = (z + 1 < s.Nz) ? u[p + pl] : cmk<double2>(0, 0);
        const double2 ud = (z > 0) ? u[p - pl] : cmk<double2>(0, 0);
        double2 zp = cadd(cmul(s.azh[z + 1], csub(uc, uu)), cmul(s.azh[z], csub(uc, ud)));
        r = cadd(r, cmul(s.az[z], zp));
    }
    r.x *= s.inv_h2; r.y *= s.inv_h2;
    const double kk = s.k2[p];
    r.x -= kk * uc.x;
    r.y -= kk * uc.y;
    return r;
}

__global__ void __launch_bounds__(256) k_apply_A(StencilArgs s, const double2* __restrict__ u,
                                                 const double2* __restrict__ f,
                                                 double2* __restrict__ out) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int l = blockIdx.y * 4 + threadIdx.y;           // row z * Ny + y
    const size_t off = (size_t)blockIdx.z * s.Nx * s.Ny * s.Nz;
    if (i >= s.Nx || l >= s.Ny * s.Nz) return;
    double2 a = stencil_at(s, u + off, l, i);
    const size_t p = off + (size_t)l * s.Nx + i;
    out[p] = f ? csub(f[p], a) : a;
}

// The same on pairs of adjacent columns (cols[2q + 1] = cols[2q] + 1): a workgroup takes 64
// rows of one pair and one right-hand side; the 4-column window i0 - 1 .. i0 + 2 of its rows
// and the two rows around them go through LDS with 64-byte contiguous loads per row (a
// thread per row and column would touch a separate cache line for every value).
__global__ void __launch_bounds__(256) k_apply_A_pairs(StencilArgs s, const int* __restrict__ cols,
                                                       const double2* __restrict__ u,
                                                       const double2* __restrict__ f,
                                                       double2* __restrict__ out) {
    __shared__ double2 T[66][4];
    const int t = threadIdx.x, c = t & 3, rr = t >> 2;
    const int i0 = cols[2 * blockIdx.y];
    const int nrow = s.Ny * s.Nz;
    const int row0 = blockIdx.x * 64;
    const size_t off = (size_t)blockIdx.z * s.Nx * nrow;
    const int x = i0 - 1 + c;
    const bool xin = x >= 0 && x < s.Nx;
    auto ld = [&](int row) {
        return (xin && row >= 0 && row < nrow) ? u[off + (size_t)row * s.Nx + x] : cmk<double2>(0, 0);
    };
    T[rr + 1][c] = ld(row0 + rr);
    if (t < 8) T[t < 4 ? 0 : 65][c] = ld(t < 4 ? row0 - 1 : row0 + 64);
    __syncthreads();
    const int row = row0 + rr;
    if (c == 0 || c == 3 || row >= nrow || !xin) return;
    const int i = x, l = row % s.Ny, z = row / s.Ny;
    const double2 uc = T[rr + 1][c];
    const double2 ue = T[rr + 1][c + 1], uw = T[rr + 1][c - 1];
    const double2 un = (l + 1 < s.Ny) ? T[rr + 2][c] : cmk<double2>(0, 0);
    const double2 us = (l > 0) ? T[rr][c] : cmk<double2>(0, 0);
    const double2 ae = s.axh[i + 1], aw = s.axh[i];
    const double2 an = s.ayh[l + 1], as = s.ayh[l];
    double2 xp = cadd(cmul(ae, csub(uc, ue)), cmul(aw, csub(uc, uw)));
    xp = cmul(s.ax[i], xp);
    double2 yp = cadd(cmul(an, csub(uc, un)), cmul(as, csub(uc, us)));
    yp = cmul(s.ay[l], yp);
    double2 r = cadd(xp, yp);
    const size_t p = off + (size_t)row * s.Nx + i;
    if (s.Nz > 1) {
        const size_t pl = (size_t)s.Ny * s.Nx;
        const double2 uu = (z + 1 < s.Nz) ? u[p + pl] : cmk<double2>(0, 0);
        const double2 ud = (z > 0) ? u[p - pl] : cmk<double2>(0, 0);
        double2 zp = cadd(cmul(s.azh[z + 1], csub(uc, uu)), cmul(s.azh[z], csub(uc, ud)));
        r = cadd(r, cmul(s.az[z], zp));
    }
    r.x *= s.inv_h2; r.y *= s.inv_h2;
    const double kk = s.k2[(size_t)row * s.Nx + i];
    r.x -= kk * uc.x;
    r.y -= kk * uc.y;
    out[p] = f ? csub(f[p], r) : r;
}

// Reduced-form stencils on interface windows (layout [nrhs][Nrow][NI][IWIN], window j holding
// the columns bw[j] .. bw[j] + IWIN - 1).  Grid (rows, right-hand sides): a workgroup takes
// one row of one right-hand side, a thread one output column (the two of a window side by
// side, then the next window), so no index needs a division.
//   MODE 0: g[c] = psi(c) - (A u)[c], c = 1, 2, with psi(c) = psi[.., 2 j + c - 2] for c = 2, 0 for c = 1
//   MODE 1: out[.., 2 j + k] = psi[.., 2 j + k] - (g[2 + k] - (A u)[2 + k]), k = 0, 1
//   MODE 2: out[.., 2 j + k] = (A u)[1 + k], k = 0, 1, with u = u + psi - gw (three window
//           fields: the concurrent sweep's v, w' and z; out on the columns beta_j - 1, beta_j)
//   MODE 3: MODE 0 with psi a full field [nrhs][Nrow][Nx] (taken at both columns c = 1, 2)
//   MODE 4: out[.., 2 j + k] = g[2 + k] - (A u)[2 + k], k = 0, 1, with g[3] = 0 (the
//           residual of the upward sweep vanishes there)
template <int MODE>
__global__ void __launch_bounds__(128) k_stencil_win(StencilArgs s, const int* __restrict__ bw,
                                                     const double* __restrict__ k2w, int NI, int nrhs,
                                                     const double2* __restrict__ u,
                                                     const double2* __restrict__ psi,
                                                     double2* __restrict__ gw, double2* __restrict__ out) {
    const int nrow = s.Ny * s.Nz;
    const size_t wrow = (size_t)NI * IWIN;
    const int row = blockIdx.x;
    const size_t rr = (size_t)blockIdx.y * nrow + row;   // r * nrow + row
    const int l = row % s.Ny, z = row / s.Ny;
    (void)nrhs;
    for (int q = threadIdx.x; q < 2 * NI; q += blockDim.x) {
        const int k = q & 1, j = q >> 1;
        const int c = (MODE == 1 || MODE == 4 ? 2 : 1) + k;
        const int i = bw[j] + c;
        const size_t b = rr * wrow + (size_t)j * IWIN + c;
        // the field at window offset d from b (MODE 2: the sum v + w' - z of three fields)
        auto U = [&](long d) {
            const size_t e = (size_t)((long)b + d);
            if (MODE == 2) return csub(cadd(u[e], psi[e]), gw[e]);
            return u[e];
        };
        const double2 uc = U(0), ue = U(1), uw = U(-1);
        const double2 un = (l + 1 < s.Ny) ? U((long)wrow) : cmk<double2>(0, 0);
        const double2 us = (l > 0) ? U(-(long)wrow) : cmk<double2>(0, 0);
        const double2 ae = s.axh[i + 1], aw = s.axh[i];
        const double2 an = s.ayh[l + 1], as = s.ayh[l];
        double2 xp = cadd(cmul(ae, csub(uc, ue)), cmul(aw, csub(uc, uw)));
        xp = cmul(s.ax[i], xp);
        double2 yp = cadd(cmul(an, csub(uc, un)), cmul(as, csub(uc, us)));
        yp = cmul(s.ay[l], yp);
        double2 a = cadd(xp, yp);
        if (s.Nz > 1) {
            const size_t pl = (size_t)s.Ny * wrow;
            const double2 uu = (z + 1 < s.Nz) ? U((long)pl) : cmk<double2>(0, 0);
            const double2 ud = (z > 0) ? U(-(long)pl) : cmk<double2>(0, 0);
            double2 zp = cadd(cmul(s.azh[z + 1], csub(uc, uu)), cmul(s.azh[z], csub(uc, ud)));
            a = cadd(a, cmul(s.az[z], zp));
        }
        a.x *= s.inv_h2; a.y *= s.inv_h2;
        const double kk = k2w[(size_t)row * wrow + (size_t)j * IWIN + c];
        a.x -= kk * uc.x;
        a.y -= kk * uc.y;
        const size_t pr = rr * (2 * (size_t)NI) + 2 * (size_t)j + (c - 2);
        if (MODE == 0) {
            const double2 f = c >= 2 ? psi[pr] : cmk<double2>(0, 0);
            gw[b] = csub(f, a);
        } else if (MODE == 3) {
            gw[b] = csub(psi[rr * (size_t)s.Nx + i], a);
        } else if (MODE == 1) {
            out[pr] = csub(psi[pr], csub(gw[b], a));
        } else if (MODE == 4) {
            out[pr] = csub(c == 2 ? gw[b] : cmk<double2>(0, 0), a);
        } else {
            out[rr * (2 * (size_t)NI) + 2 * (size_t)j + k] = a;
        }
    }
}

StencilArgs stencil_args(const DevTables& t, const Geom& g) {
    StencilArgs s;
    s.k2 = t.k2; s.ax = t.ax; s.axh = t.axh; s.ay = t.ay; s.ayh = t.ayh;
    s.az = t.az; s.azh = t.azh;
    s.Nx = g.Nx; s.Ny = g.Ny; s.Nz = g.Nz; s.inv_h2 = 1.0 / (g.h * g.h);
    return s;
}

// ---------------------------------------------------------------- GMRES vectors
constexpr int NV = 8;   // basis vectors per pass of the dot kernel

__device__ inline double2 block_sum(double2 v, double2* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) sh[t] = cadd(sh[t], sh[t + o]);
        __syncthreads();
    }
    double2 r = sh[0];
    __syncthreads();
    return r;
}

// partial[(b * nrhs + r) * nvec + i] = sum over block b's slice of conj(V_i[r]) w[r]
__global__ void __launch_bounds__(256) k_dots(const double2* __restrict__ V, int nvec,
                                              const double2* __restrict__ w, int nrhs, long n,
                                              double2* __restrict__ partial) {
    __shared__ double2 sh[256];
    const int b = blockIdx.x, r = blockIdx.y, nb = gridDim.x;
    const long per = (n + nb - 1) / nb;
    const long lo = (long)b * per, hi = min(n, lo + per);
    const size_t vs = (size_t)nrhs * n;
    const double2* wr = w + (size_t)r * n;
    for (int i0 = 0; i0 < nvec; i0 += NV) {
        double2 acc[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] = cmk<double2>(0, 0);
        for (long p = lo + threadIdx.x; p < hi; p += 256) {
            const double2 wv = wr[p];
#pragma unroll
            for (int q = 0; q < NV; ++q)
                if (i0 + q < nvec) {
                    const double2 v = V[(size_t)(i0 + q) * vs + (size_t)r * n + p];
                    const double2 m = cconjmul(v, wv);
                    acc[q] = cadd(acc[q], m);
                }
        }
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            if (i0 + q >= nvec) break;
            const double2 s = block_sum(acc[q], sh);
            if (threadIdx.x == 0) partial[((size_t)b * nrhs + r) * nvec + i0 + q] = s;
        }
    }
}

__global__ void k_reduce_partials(const double2* __restrict__ partial, int nb, int m,
                                  double2* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;   // j = r * nvec + i
    if (j >= m) return;
    double2 s = cmk<double2>(0, 0);
    for (int b = 0; b < nb; ++b) s = cadd(s, partial[(size_t)b * m + j]);
    out[j] = s;
}

// w[r] -= sum_i h[r][i] V_i[r]
// grid (blocks, right-hand sides): blockIdx.y is the right-hand side (no division per element)
__global__ void k_update(const double2* __restrict__ V, int nvec, const double2* __restrict__ h,
                         double2* __restrict__ w, int nrhs, long n) {
    const size_t tot = (size_t)nrhs * n;
    const int r = blockIdx.y;
    for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x) {
        const size_t q = (size_t)r * n + p;
        double2 acc = w[q];
        for (int i = 0; i < nvec; ++i) acc = csub(acc, cmul(h[r * nvec + i], V[(size_t)i * tot + q]));
        w[q] = acc;
    }
}

__global__ void __launch_bounds__(256) k_norms(const double2* __restrict__ w, int nrhs, long n,
                                               double* __restrict__ partial) {
    __shared__ double2 sh[256];
    const int b = blockIdx.x, r = blockIdx.y, nb = gridDim.x;
    const long per = (n + nb - 1) / nb;
    const long lo = (long)b * per, hi = min(n, lo + per);
    const double2* wr = w + (size_t)r * n;
    double acc = 0.0;
    for (long p = lo + threadIdx.x; p < hi; p += 256) {
        const double2 v = wr[p];
        acc = fma(v.x, v.x, acc);
        acc = fma(v.y, v.y, acc);
    }
    const double2 s = block_sum(cmk<double2>(acc, 0.0), sh);
    if (threadIdx.x == 0) partial[(size_t)b * nrhs + r] = s.x;
}

__global__ void k_reduce_norms(const double* __restrict__ partial, int nb, int nrhs,
                               double* __restrict__ out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[(size_t)b * nrhs + r];
    out[r] = sqrt(s);
}

__global__ void k_scale(const double2* __restrict__ w, const double* __restrict__ nrm,
                        double2* __restrict__ out, int nrhs, long n) {
    const size_t tot = (size_t)nrhs * n;
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < tot;
         q += (size_t)gridDim.x * blockDim.x) {
        const double d = nrm[q / n];
        const double2 v = w[q];
        out[q] = d > 0.0 ? cmk<double2>(v.x / d, v.y / d) : cmk<double2>(0.0, 0.0);
    }
}

__global__ void k_lincomb(const double2* __restrict__ V, int nvec, const double2* __restrict__ y,
                          double2* __restrict__ out, int nrhs, long n, int accumulate) {
    const size_t tot = (size_t)nrhs * n;
    const int r = blockIdx.y;
    for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x) {
        const size_t q = (size_t)r * n + p;
        double2 acc = accumulate ? out[q] : cmk<double2>(0, 0);
        for (int i = 0; i < nvec; ++i) acc = cadd(acc, cmul(y[r * nvec + i], V[(size_t)i * tot + q]));
        out[q] = acc;
    }
}

__global__ void k_gather_cols(const double2* __restrict__ field, const int* __restrict__ cols,
                              int ncols, int nrhs, int Ny, int Nx, double2* __restrict__ red) {
    const size_t tot = (size_t)nrhs * Ny * ncols;
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < tot;
         q += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(q % ncols);
        const size_t rl = q / ncols;          // r * Ny + l
        red[q] = field[rl * Nx + cols[k]];
    }
}

__global__ void k_scatter_cols(const double2* __restrict__ red, const int* __restrict__ cols,
                               int ncols, int nrhs, int Ny, int Nx, double2* __restrict__ field, int add) {
    const size_t tot = (size_t)nrhs * Ny * ncols;
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < tot;
         q += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(q % ncols);
        const size_t rl = q / ncols;
        double2* p = field + rl * Nx + cols[k];
        *p = add ? cadd(*p, red[q]) : red[q];
    }
}

// entries c0 .. c0 + n - 1 of every row's first window (window fields [nrows][wrow]) set to 0
__global__ void k_clear_win_cols(double2* __restrict__ win, long nrows, long wrow, int c0, int n) {
    const long tot = nrows * n;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < tot; q += (long)gridDim.x * blockDim.x)
        win[(q / n) * wrow + c0 + q % n] = cmk<double2>(0, 0);
}

// out = x + y + z (x or z may be null: treated as zero)
__global__ void k_sum3(const double2* __restrict__ x, const double2* __restrict__ y,
                       const double2* __restrict__ z, double2* __restrict__ out, long n, double zs) {
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        double2 v = y[q];
        if (x) v = cadd(x[q], v);
        if (z) { v.x += zs * z[q].x; v.y += zs * z[q].y; }
        out[q] = v;
    }
}

// Robin data: out[r][row] = (vo - rho[row] vi)[r][row] * ih2
__global__ void k_robin_data(const double2* __restrict__ vo, const double2* __restrict__ vi,
                             const double2* __restrict__ rho, double2* __restrict__ out, long n, long Nrow,
                             double ih2) {
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const double2 d = csub(vo[q], cmul(rho[q % Nrow], vi[q]));
        out[q] = make_double2(d.x * ih2, d.y * ih2);
    }
}

inline unsigned grid_for(size_t tot) {
    size_t b = (tot + 255) / 256;
    return (unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

}  // namespace

int dots_blocks(long n) {
    long nb = (n + 8191) / 8192;
    if (nb < 1) nb = 1;
    if (nb > 256) nb = 256;
    return (int)nb;
}

hipError_t launch_apply_A(const DevTables& t, const Geom& g, int nrhs, const double2* u,
                          const double2* f, double2* out, hipStream_t st) {
    StencilArgs s = stencil_args(t, g);
    dim3 grid((g.Nx + 63) / 64, (unsigned)((g.Nrow() + 3) / 4), nrhs);
    hipLaunchKernelGGL(k_apply_A, grid, dim3(64, 4), 0, st, s, u, f, out);
    return hipGetLastError();
}

hipError_t launch_apply_A_pairs(const DevTables& t, const Geom& g, int nrhs, const int* cols,
                               int npairs, const double2* u, const double2* f, double2* out,
                               hipStream_t st) {
    if (npairs <= 0) return hipSuccess;
    StencilArgs s = stencil_args(t, g);
    dim3 grid((unsigned)((g.Nrow() + 63) / 64), npairs, nrhs);
    hipLaunchKernelGGL(k_apply_A_pairs, grid, dim3(256), 0, st, s, cols, u, f, out);
    return hipGetLastError();
}

hipError_t launch_stencil_win(int mode, const DevTables& t, const Geom& g, int nrhs, const double2* u,
                              const double2* psi, double2* gw, double2* out, hipStream_t st) {
    const int NI = g.J - 1;
    if (NI <= 0) return hipSuccess;
    StencilArgs s = stencil_args(t, g);
    const dim3 grid((unsigned)g.Nrow(), (unsigned)nrhs);
    if (mode == 0)
        hipLaunchKernelGGL(k_stencil_win<0>, grid, dim3(128), 0, st, s, t.bw, t.k2w, NI, nrhs, u, psi, gw, out);
    else if (mode == 1)
        hipLaunchKernelGGL(k_stencil_win<1>, grid, dim3(128), 0, st, s, t.bw, t.k2w, NI, nrhs, u, psi, gw, out);
    else if (mode == 3)
        hipLaunchKernelGGL(k_stencil_win<3>, grid, dim3(128), 0, st, s, t.bw, t.k2w, NI, nrhs, u, psi, gw, out);
    else if (mode == 4)
        hipLaunchKernelGGL(k_stencil_win<4>, grid, dim3(128), 0, st, s, t.bw, t.k2w, NI, nrhs, u, psi, gw, out);
    else
        hipLaunchKernelGGL(k_stencil_win<2>, grid, dim3(128), 0, st, s, t.bw, t.k2w, NI, nrhs, u, psi, gw, out);
    return hipGetLastError();
}

hipError_t launch_dots(const double2* V, int nvec, const double2* w, int nrhs, long n,
                       double2* partial, int nblk, double2* out, hipStream_t st) {
    hipLaunchKernelGGL(k_dots, dim3(nblk, nrhs), dim3(256), 0, st, V, nvec, w, nrhs, n, partial);
    const int m = nrhs * nvec;
    hipLaunchKernelGGL(k_reduce_partials, dim3((m + 255) / 256), dim3(256), 0, st, partial, nblk,
                       m, out);
    return hipGetLastError();
}

hipError_t launch_update(const double2* V, int nvec, const double2* h, double2* w, int nrhs,
                         long n, hipStream_t st) {
    const unsigned bx = std::max(1u, grid_for((size_t)nrhs * n) / (unsigned)nrhs);
    hipLaunchKernelGGL(k_update, dim3(bx, nrhs), dim3(256), 0, st, V, nvec, h, w, nrhs, n);
    return hipGetLastError();
}

hipError_t launch_norms(const double2* w, int nrhs, long n, double* partial, int nblk,
                        double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_norms, dim3(nblk, nrhs), dim3(256), 0, st, w, nrhs, n, partial);
    hipLaunchKernelGGL(k_reduce_norms, dim3((nrhs + 255) / 256), dim3(256), 0, st, partial, nblk,
                       nrhs, out);
    return hipGetLastError();
}

hipError_t launch_scale(const double2* w, const double* nrm, double2* out, int nrhs, long n,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_scale, dim3(grid_for((size_t)nrhs * n)), dim3(256), 0, st, w, nrm, out,
                       nrhs, n);
    return hipGetLastError();
}

hipError_t launch_lincomb(const double2* V, int nvec, const double2* y, double2* out,
                          int nrhs, long n, int accumulate, hipStream_t st) {
    const unsigned bx = std::max(1u, grid_for((size_t)nrhs * n) / (unsigned)nrhs);
    hipLaunchKernelGGL(k_lincomb, dim3(bx, nrhs), dim3(256), 0, st, V, nvec, y, out, nrhs, n, accumulate);
    return hipGetLastError();
}

hipError_t launch_gather_cols(const double2* field, const int* cols, int ncols, int nrhs,
                              int Ny, int Nx, double2* red, hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_cols, dim3(grid_for((size_t)nrhs * Ny * ncols)), dim3(256), 0, st,
                       field, cols, ncols, nrhs, Ny, Nx, red);
    return hipGetLastError();
}

hipError_t launch_scatter_cols(const double2* red, const int* cols, int ncols, int nrhs,
                               int Ny, int Nx, double2* field, hipStream_t st, bool add) {
    if (ncols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_cols, dim3(grid_for((size_t)nrhs * Ny * ncols)), dim3(256), 0, st,
                       red, cols, ncols, nrhs, Ny, Nx, field, add ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_clear_win_cols(double2* win, long nrows, long wrow, int c0, int n, hipStream_t st) {
    if (nrows <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear_win_cols, dim3(grid_for((size_t)nrows * n)), dim3(256), 0, st, win, nrows, wrow,
                       c0, n);
    return hipGetLastError();
}

hipError_t launch_sum3(const double2* x, const double2* y, const double2* z, double2* out, long n,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_sum3, dim3(grid_for((size_t)n)), dim3(256), 0, st, x, y, z, out, n, 1.0);
    return hipGetLastError();
}

hipError_t launch_robin_data(const double2* vo, const double2* vi, const double2* rho, double2* out, int nrhs,
                             long Nrow, double ih2, hipStream_t st) {
    const long n = (long)nrhs * Nrow;
    hipLaunchKernelGGL(k_robin_data, dim3(grid_for((size_t)n)), dim3(256), 0, st, vo, vi, rho, out, n, Nrow, ih2);
    return hipGetLastError();
}

hipError_t launch_sum_diff(const double2* x, const double2* y, const double2* z, double2* out, long n,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_sum3, dim3(grid_for((size_t)n)), dim3(256), 0, st, x, y, z, out, n, -1.0);
    return hipGetLastError();
}

}  // namespace helm

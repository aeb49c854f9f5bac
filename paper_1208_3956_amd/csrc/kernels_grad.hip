// Misfit and adjoint-state gradient with respect to the squared slowness m = 1/c^2.
//
// The paper has no gradient; this is the differentiation form of its solver.  With sources
// f_s, receivers R (padded-grid points) and data d_s:
//     J(m) = 1/2 sum_s |R u_s - d_s|^2,          A(m) u_s = f_s,
//     dJ/dm_p = omega^2 Re sum_s sum_{q -> p} conj(lambda_s[q]) u_s[q],   A^H lambda_s = R^T r_s,
// r_s = R u_s - d_s, where q runs over the padded points whose medium is copied from the
// interior point p (the outer PML continues the nearest interior value).  Only the -k^2 u
// term of A depends on m (k^2 = omega^2 m).
//
// The PML operator of Sec. 2.2 is A = D S with D = alpha_x(x_i) alpha_y(y_l) and S complex
// symmetric, so A^H = conj(S) conj(D) and A^H lambda = q  <=>  A (D conj(lambda)) = D conj(q).
// The adjoint field is therefore one more solve with the same factors: z = A^{-1} D conj(q),
// conj(lambda) = z / D, and the gradient term is omega^2 Re(z u / D).
#include "helm_internal.hpp"

namespace helm {
namespace {

__device__ inline double2 cd_mul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// r[s][k] = u[s][rec[k]] - d[s][k]
__global__ void k_rec_residual(const double2* __restrict__ u, long field, const long* __restrict__ rec,
                               int nrec, const double2* __restrict__ d, int nsrc, double2* __restrict__ r) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)nsrc * nrec) return;
    const int s = (int)(i / nrec), k = (int)(i % nrec);
    const double2 a = u[(size_t)s * field + rec[k]], b = d[i];
    r[i] = make_double2(a.x - b.x, a.y - b.y);
}

// 1/2 sum |r|^2 in one workgroup: fixed per-thread strides and a fixed tree (deterministic)
__global__ void __launch_bounds__(256) k_half_sumsq(const double2* __restrict__ r, long n,
                                                    double* __restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (long i = threadIdx.x; i < n; i += 256) acc += r[i].x * r[i].x + r[i].y * r[i].y;
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = 0.5 * red[0];
}

// Adjoint right-hand side on the receiver points: Q[s][p] = D[p] conj(sum_{k: rec[k]=p} r[s][k]).
// Receivers are grouped by point on the host (upt[j] = point, [ustart[j], ustart[j+1]) the
// positions k of that point in the receiver list, in order), so repeated receivers add up
// without atomics.  Q must be zero elsewhere.
__global__ void k_adjoint_rhs(const double2* __restrict__ r, int nrec, int nsrc,
                              const long* __restrict__ upt, const int* __restrict__ ustart,
                              const int* __restrict__ uidx, int nu, const double2* __restrict__ ax,
                              const double2* __restrict__ ay, int Nx, long field,
                              double2* __restrict__ Q) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)nsrc * nu) return;
    const int s = (int)(i / nu), j = (int)(i % nu);
    double2 acc = make_double2(0.0, 0.0);
    for (int t = ustart[j]; t < ustart[j + 1]; ++t) {
        const double2 v = r[(size_t)s * nrec + uidx[t]];
        acc.x += v.x;
        acc.y += v.y;
    }
    const long p = upt[j];
    const double2 D = cd_mul(ax[p % Nx], ay[p / Nx]);
    Q[(size_t)s * field + p] = cd_mul(D, make_double2(acc.x, -acc.y));
}

// grad[l][i] = omega^2 sum_s sum over the padded points (x, y) whose medium is taken from the
// interior point (i, l) of Re(z u / D).  Interior points on an edge of the interior collect the
// outer-PML points behind them (a w_out + 1 long run; corners a square).
__global__ void __launch_bounds__(256) k_grad_m(const double2* __restrict__ u, const double2* __restrict__ z,
                                                int nsrc, const double2* __restrict__ ax,
                                                const double2* __restrict__ ay, int nx, int ny, int wout,
                                                double omega2, double* __restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (i >= nx || l >= ny) return;
    const int Nx = nx + 2 * wout, Ny = ny + 2 * wout;
    const int x0 = i == 0 ? 0 : i + wout, x1 = i == nx - 1 ? Nx - 1 : i + wout;
    const int y0 = l == 0 ? 0 : l + wout, y1 = l == ny - 1 ? Ny - 1 : l + wout;
    const size_t field = (size_t)Nx * Ny;
    double acc = 0.0;
    for (int y = y0; y <= y1; ++y) {
        for (int x = x0; x <= x1; ++x) {
            const double2 D = cd_mul(ax[x], ay[y]);
            const double dn = D.x * D.x + D.y * D.y;
            const double2 Dinv = make_double2(D.x / dn, -D.y / dn);
            const size_t p = (size_t)y * Nx + x;
            for (int s = 0; s < nsrc; ++s) {
                const double2 zu = cd_mul(z[s * field + p], u[s * field + p]);
                acc += zu.x * Dinv.x - zu.y * Dinv.y;
            }
        }
    }
    grad[(size_t)l * nx + i] = omega2 * acc;
}

inline unsigned blocks_for(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_rec_residual(const double2* u, long field, const long* rec, int nrec,
                               const double2* d, int nsrc, double2* r, hipStream_t st) {
    hipLaunchKernelGGL(k_rec_residual, dim3(blocks_for((long)nsrc * nrec)), dim3(256), 0, st, u, field,
                       rec, nrec, d, nsrc, r);
    return hipGetLastError();
}

hipError_t launch_half_sumsq(const double2* r, long n, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_half_sumsq, dim3(1), dim3(256), 0, st, r, n, out);
    return hipGetLastError();
}

hipError_t launch_adjoint_rhs(const double2* r, int nrec, int nsrc, const long* upt, const int* ustart,
                              const int* uidx, int nu, const DevTables& t, const Geom& g, double2* Q,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_adjoint_rhs, dim3(blocks_for((long)nsrc * nu)), dim3(256), 0, st, r, nrec, nsrc,
                       upt, ustart, uidx, nu, t.ax, t.ay, g.Nx, (long)g.Nx * g.Ny, Q);
    return hipGetLastError();
}

hipError_t launch_grad_m(const double2* u, const double2* z, int nsrc, const DevTables& t,
                         const Geom& g, double* grad, hipStream_t st) {
    dim3 grid((g.nx + 255) / 256, g.ny);
    hipLaunchKernelGGL(k_grad_m, grid, dim3(256), 0, st, u, z, nsrc, t.ax, t.ay, g.nx, g.ny, g.wout,
                       g.omega * g.omega, grad);
    return hipGetLastError();
}

}  // namespace helm

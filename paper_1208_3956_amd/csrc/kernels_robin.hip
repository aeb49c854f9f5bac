// Kernels of the concurrent sweeps with Robin transmission (Sec. 3.1, with the Robin
// conditions of Sec. 4.4): the right-hand side of one subdomain problem with two-sided data,
// and the assembly of v from the subdomains' latest solutions.
#include "helm_internal.hpp"

namespace helm {

namespace {

// out[r][l][q], q < W: f on the core columns [c0, c1) of the subdomain (strip-local), plus on
// the first column the Robin data (V_o - rho_l V_i) / h^2 of the left neighbour's latest
// solution L (global columns lo - 1 outside, lo inside) and on the last column that of the
// right neighbour's R (columns hi outside, hi - 1 inside); a null neighbour adds nothing.
__global__ void k_robin_rhs(const double2* __restrict__ f, const double2* __restrict__ L,
                            const double2* __restrict__ R, const double2* __restrict__ rho_l,
                            const double2* __restrict__ rho_r, double2* __restrict__ out, int nrhs,
                            int Nrow, int Nx, int lo, int W, int c0, int c1, double ih2) {
    const long field = (long)Nrow * Nx;
    const long n = (long)nrhs * Nrow * W;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const int q = (int)(e % W);
        const long rl = e / W;                       // r * Nrow + l
        const int l = (int)(rl % Nrow);
        const long r = rl / Nrow;
        const double2* frow = f + r * field + (long)l * Nx;
        double2 v = (q >= c0 && q < c1) ? frow[lo + q] : make_double2(0.0, 0.0);
        if (q == 0 && L) {
            const double2* row = L + r * field + (long)l * Nx;
            const double2 d = csub(row[lo - 1], cmul(rho_l[l], row[lo]));
            v.x += d.x * ih2;
            v.y += d.y * ih2;
        }
        if (q == W - 1 && R) {
            const double2* row = R + r * field + (long)l * Nx;
            const int hi = lo + W;
            const double2 d = csub(row[hi], cmul(rho_r[l], row[hi - 1]));
            v.x += d.x * ih2;
            v.y += d.y * ih2;
        }
        out[e] = v;
    }
}

// out[r][l][x] = (par[x] ? O : E)[r][l][x]
__global__ void k_parity_pick(const double2* __restrict__ E, const double2* __restrict__ O,
                              const int* __restrict__ par, double2* __restrict__ out, long n, int Nx) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        out[e] = par[e % Nx] ? O[e] : E[e];
}

inline unsigned blocks_for(long n) {
    long b = (n + 255) / 256;
    return (unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

}  // namespace

hipError_t launch_robin_rhs(const double2* f, const double2* L, const double2* R, const double2* rho_l,
                            const double2* rho_r, double2* out, int nrhs, int Nrow, int Nx, int lo, int W,
                            int c0, int c1, double ih2, hipStream_t st) {
    const long n = (long)nrhs * Nrow * W;
    hipLaunchKernelGGL(k_robin_rhs, dim3(blocks_for(n)), dim3(256), 0, st, f, L, R, rho_l, rho_r, out, nrhs,
                       Nrow, Nx, lo, W, c0, c1, ih2);
    return hipGetLastError();
}

hipError_t launch_parity_pick(const double2* E, const double2* O, const int* par, double2* out, int nrhs,
                              long Nrow, int Nx, hipStream_t st) {
    const long n = (long)nrhs * Nrow * Nx;
    hipLaunchKernelGGL(k_parity_pick, dim3(blocks_for(n)), dim3(256), 0, st, E, O, par, out, n, Nx);
    return hipGetLastError();
}

}  // namespace helm

// Strip solves x = A^(j)^{-1} r with the chunked block-LU factors (the subdomain solves of
// eqs. solve_upward / solve_downward, Sec. 2.1-2.2), for a panel of right-hand sides.
//
// With chunks I_c (interior rows) and separators s_c (see kernels_factor.hip):
//   phase A  (all chunks in parallel)  y_I = A_I^{-1} r_I by forward / backward block
//            substitution  z_l = G_l (r_l - c_l z_{l-1}),  y_l = z_l - b_l G_l y_{l+1}
//   phase B  (one sweep over separators) r^_c = r_s - c_s y_{s-1} - b_s y_{s+1};
//            z'_c = G'_c (r^_c - L_c z'_{c-1});  x_s = z'_c - U'_c x_{s'}
//   phase C  (all rows in parallel)     x_l = y_l - X~_l x_{s above} - Y~_l x_{s below}
// Phase A gathers the right-hand side (restriction of a field to the strip plus the
// two-column transmission source of Sec. 2.2); phase C scatters the requested columns of
// x into the output field and writes the two trace columns the next strip needs.
//
// Arithmetic is in T (float or double complex); gathered and scattered fields are FP64.
#include "helm_internal.hpp"

namespace helm {

namespace {

constexpr int NT = 256;

template <typename T>
struct SolveArgs {
    const cplx<T>* F;     // factors of the strip: [Ny][NSLOT][WP*WP]
    cplx<T>* Yw;          // workspace [nrhs][Ny][WP]
    const double2* cy;
    const double2* by;
    IOSpec io;
    int Ny, W, m, P, nrhs;
};

template <typename T>
__device__ inline cplx<T> gather(const IOSpec& io, int r, int l, int q, int Ny) {
    double2 v = cmk<double2>(0.0, 0.0);
    if (q >= io.src_lo && q < io.src_hi)
        v = io.src[(size_t)r * io.src_rs + (size_t)l * io.src_ls + (q + io.src_off)];
    if (io.q_t >= 0 && (q == io.q_t || q == io.q_t + 1)) {
        const double2 ta = io.trA[(size_t)r * Ny + l], tb = io.trB[(size_t)r * Ny + l];
        v.x += io.coef * (tb.x - ta.x);
        v.y += io.coef * (tb.y - ta.y);
    }
    return ccast<cplx<T>>(v);
}

template <typename T>
__device__ inline const cplx<T>* fslot(const SolveArgs<T>& a, int l, int sl) {
    return a.F + ((size_t)l * NSLOT + sl) * BLK;
}

// acc[u] += sum_k M(i,k) vin[k][g + 4u] over k < W  (M column-major, ld WP)
template <typename T, int R>
__device__ inline void matvec_acc(cplx<T> (&acc)[R / 4], const cplx<T>* __restrict__ M,
                                  const cplx<T> (*vin)[R], int W, int i, int g) {
    constexpr int U = R / 4;
    for (int k = 0; k < W; ++k) {
        const cplx<T> mk = M[(size_t)k * WP + i];
#pragma unroll
        for (int u = 0; u < U; ++u) cfma(acc[u], mk, vin[k][g + 4 * u]);
    }
}

// ---------------------------------------------------------------- phase A
template <typename T, int R>
__global__ void __launch_bounds__(NT) k_phase_a(SolveArgs<T> a) {
    using V = cplx<T>;
    constexpr int U = R / 4;
    __shared__ V vin[WP][R];
    const int t = threadIdx.x, i = t & (WP - 1), g = t >> 6;
    const int c = blockIdx.x, rbase = blockIdx.y * R;
    const int r0 = c * a.m;
    const int r1 = (c < a.P - 1) ? c * a.m + a.m - 1 : a.Ny;
    const V zero = cmk<V>(0, 0);
    V z[U];
#pragma unroll
    for (int u = 0; u < U; ++u) z[u] = zero;

    for (int l = r0; l < r1; ++l) {
        const V cl = ccast<V>(a.cy[l]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = rbase + g + 4 * u;
            V v = zero;
            if (r < a.nrhs && i < a.W) {
                v = gather<T>(a.io, r, l, i, a.Ny);
                if (l > r0) v = csub(v, cmul(cl, z[u]));
            }
            vin[i][g + 4 * u] = v;
        }
        __syncthreads();
        V acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = zero;
        matvec_acc<T, R>(acc, fslot(a, l, 0), vin, a.W, i, g);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = rbase + g + 4 * u;
            z[u] = acc[u];
            if (r < a.nrhs) a.Yw[((size_t)r * a.Ny + l) * WP + i] = acc[u];
        }
        __syncthreads();
    }
    // backward: y_{r1-1} = z_{r1-1};  y_l = z_l - b_l G_l y_{l+1}
    for (int l = r1 - 2; l >= r0; --l) {
#pragma unroll
        for (int u = 0; u < U; ++u) vin[i][g + 4 * u] = z[u];
        __syncthreads();
        V acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = zero;
        matvec_acc<T, R>(acc, fslot(a, l, 0), vin, a.W, i, g);
        const V bl = ccast<V>(a.by[l]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = rbase + g + 4 * u;
            if (r < a.nrhs) {
                V* p = a.Yw + ((size_t)r * a.Ny + l) * WP + i;
                const V y = csub(*p, cmul(bl, acc[u]));
                *p = y;
                z[u] = y;
            } else {
                z[u] = zero;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- phase B
template <typename T, int R>
__global__ void __launch_bounds__(NT) k_phase_b(SolveArgs<T> a) {
    using V = cplx<T>;
    constexpr int U = R / 4;
    __shared__ V vin[WP][R];
    const int t = threadIdx.x, i = t & (WP - 1), g = t >> 6;
    const int rbase = blockIdx.x * R;
    const V zero = cmk<V>(0, 0);
    V z[U];
#pragma unroll
    for (int u = 0; u < U; ++u) z[u] = zero;

    for (int c = 0; c + 1 < a.P; ++c) {
        const int s = c * a.m + a.m - 1;
        const V cs = ccast<V>(a.cy[s]), bs = ccast<V>(a.by[s]);
        V rh[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = rbase + g + 4 * u;
            V v = zero;
            if (r < a.nrhs && i < a.W) {
                v = gather<T>(a.io, r, s, i, a.Ny);
                const V yu = a.Yw[((size_t)r * a.Ny + (s - 1)) * WP + i];
                const V yd = a.Yw[((size_t)r * a.Ny + (s + 1)) * WP + i];
                v = csub(v, cmul(cs, yu));
                v = csub(v, cmul(bs, yd));
            }
            rh[u] = v;
        }
        if (c >= 1) {
#pragma unroll
            for (int u = 0; u < U; ++u) vin[i][g + 4 * u] = z[u];
            __syncthreads();
            V acc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) acc[u] = zero;
            matvec_acc<T, R>(acc, fslot(a, s, 1), vin, a.W, i, g);
#pragma unroll
            for (int u = 0; u < U; ++u) rh[u] = csub(rh[u], acc[u]);
            __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < U; ++u) vin[i][g + 4 * u] = rh[u];
        __syncthreads();
        V acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = zero;
        matvec_acc<T, R>(acc, fslot(a, s, 0), vin, a.W, i, g);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = rbase + g + 4 * u;
            z[u] = acc[u];
            if (r < a.nrhs) a.Yw[((size_t)r * a.Ny + s) * WP + i] = acc[u];
        }
        __syncthreads();
    }
    // backward over separators: x_c = z'_c - U'_c x_{c+1}
    for (int c = a.P - 3; c >= 0; --c) {
        const int s = c * a.m + a.m - 1;
#pragma unroll
        for (int u = 0; u < U; ++u) vin[i][g + 4 * u] = z[u];
        __syncthreads();
        V acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = zero;
        matvec_acc<T, R>(acc, fslot(a, s, 2), vin, a.W, i, g);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = rbase + g + 4 * u;
            if (r < a.nrhs) {
                V* p = a.Yw + ((size_t)r * a.Ny + s) * WP + i;
                const V x = csub(*p, acc[u]);
                *p = x;
                z[u] = x;
            } else {
                z[u] = zero;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- phase C
template <typename T, int R>
__global__ void __launch_bounds__(NT) k_phase_c(SolveArgs<T> a) {
    using V = cplx<T>;
    constexpr int U = R / 4;
    __shared__ V va[WP][R];
    __shared__ V vb[WP][R];
    const int t = threadIdx.x, i = t & (WP - 1), g = t >> 6;
    const int l = blockIdx.x, rbase = blockIdx.y * R;
    const int c = l / a.m;
    const bool is_sep = (c < a.P - 1) && (l == c * a.m + a.m - 1);
    const bool top = !is_sep && c > 0;
    const bool bot = !is_sep && c < a.P - 1;
    const V zero = cmk<V>(0, 0);
    V x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int r = rbase + g + 4 * u;
        x[u] = (r < a.nrhs) ? a.Yw[((size_t)r * a.Ny + l) * WP + i] : zero;
        V xa = zero, xb = zero;
        if (r < a.nrhs) {
            if (top) xa = a.Yw[((size_t)r * a.Ny + (c * a.m - 1)) * WP + i];
            if (bot) xb = a.Yw[((size_t)r * a.Ny + (c * a.m + a.m - 1)) * WP + i];
        }
        va[i][g + 4 * u] = xa;
        vb[i][g + 4 * u] = xb;
    }
    __syncthreads();
    if (top || bot) {
        V acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = zero;
        if (top) matvec_acc<T, R>(acc, fslot(a, l, 1), va, a.W, i, g);
        if (bot) matvec_acc<T, R>(acc, fslot(a, l, 2), vb, a.W, i, g);
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = csub(x[u], acc[u]);
    }
    const IOSpec& io = a.io;
    const bool o0 = i >= io.o_lo[0] && i < io.o_hi[0];
    const bool o1 = i >= io.o_lo[1] && i < io.o_hi[1];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int r = rbase + g + 4 * u;
        if (r >= a.nrhs || i >= a.W) continue;
        const double2 xv = ccast<double2>(x[u]);
        if ((o0 || o1) && io.dst) {
            double2* p = io.dst + (size_t)r * io.dst_rs + (size_t)l * io.dst_ls + (i + io.dst_off);
            *p = io.accumulate ? cadd(*p, xv) : xv;
        }
        if (i == io.qo0 && io.tro0) io.tro0[(size_t)r * a.Ny + l] = xv;
        if (i == io.qo1 && io.tro1) io.tro1[(size_t)r * a.Ny + l] = xv;
    }
}

template <typename T, int R>
hipError_t run(const SolveArgs<T>& a, hipStream_t st, KTimer* kt) {
    const int RG = (a.nrhs + R - 1) / R;
    if (kt) kt->begin(K_PHASE_A, st);
    hipLaunchKernelGGL((k_phase_a<T, R>), dim3(a.P, RG), dim3(NT), 0, st, a);
    if (kt) kt->end(K_PHASE_A, st);
    if (a.P > 1) {
        if (kt) kt->begin(K_PHASE_B, st);
        hipLaunchKernelGGL((k_phase_b<T, R>), dim3(RG), dim3(NT), 0, st, a);
        if (kt) kt->end(K_PHASE_B, st);
    }
    if (kt) kt->begin(K_PHASE_C, st);
    hipLaunchKernelGGL((k_phase_c<T, R>), dim3(a.Ny, RG), dim3(NT), 0, st, a);
    if (kt) kt->end(K_PHASE_C, st);
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_strip_solve(const DevTables& t, const Geom& g, const Chunks& ch, int s,
                              const cplx<T>* F, cplx<T>* Yw, int nrhs, const IOSpec& io,
                              hipStream_t st, KTimer* kt) {
    SolveArgs<T> a;
    a.F = F + (size_t)s * g.Ny * NSLOT * BLK;
    a.Yw = Yw;
    a.cy = t.cy;
    a.by = t.by;
    a.io = io;
    a.Ny = g.Ny;
    a.W = g.strips[s].W;
    a.m = ch.m;
    a.P = ch.P;
    a.nrhs = nrhs;
    if (nrhs <= 4) return run<T, 4>(a, st, kt);
    return run<T, 16>(a, st, kt);
}

template hipError_t launch_strip_solve<float>(const DevTables&, const Geom&, const Chunks&, int,
                                              const float2*, float2*, int, const IOSpec&,
                                              hipStream_t, KTimer*);
template hipError_t launch_strip_solve<double>(const DevTables&, const Geom&, const Chunks&, int,
                                               const double2*, double2*, int, const IOSpec&,
                                               hipStream_t, KTimer*);

}  // namespace helm

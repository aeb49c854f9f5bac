// Strip solves x = A^(j)^{-1} r with the chunked block-LU factors (the subdomain solves of
// eqs. solve_upward / solve_downward, Sec. 2.1-2.2), for a panel of right-hand sides.
//
// With chunks I_c (interior rows) and separators s_c (see kernels_factor.hip):
//   phase A   (chunks x rhs groups)  y_I = A_I^{-1} r_I by forward / backward block
//             substitution  z_l = G_l (r_l - c_l z_{l-1}),  y_l = z_l - b_l G_l y_{l+1}
//   phase B0  (separators x rhs)     a_c = G'_c r^_c,  r^_c = r_s - c_s y_{s-1} - b_s y_{s+1}
//   phase B   (one workgroup per rhs) z'_c = a_c - K_c z'_{c-1};  x_s = z'_c - U'_c x_{s'}
//   phase C   (rows x rhs groups)    x_l = y_l - X~_l x_{s above} - Y~_l x_{s below}
// Phase A (and B0) gather the right-hand side (a field restricted to the strip plus the
// two-column transmission source of Sec. 2.2); phase C scatters the requested columns of x
// and the two trace columns the next strip needs.  When only a few columns are requested
// (the reduced form), phase C computes just those from compact copies of the spike rows.
//
// The chains of phases A and B read the next factor block from global memory into
// registers while the current block (in LDS) is applied, then store it to the other LDS
// buffer: the latency of the block loads stays off the dependency chain.
//
// Arithmetic is in T (float or double complex); gathered and scattered fields are FP64.
#include "helm_internal.hpp"

#include <type_traits>

namespace helm {

namespace {

constexpr int NT = 256;

template <typename T>
struct SolveArgs {
    const cplx<T>* F;     // factors of the strip: [Ny][NSLOT][WP*WP]
    const cplx<T>* Fc;    // compact spike rows of the strip: [Ny][2][8][WP] (reduced phase C)
    const int* tcol;      // 8 strip-local columns of the compact rows (-1 = unused)
    const cplx<T>* Fs;    // separator propagators of the strip: [P-1][2][WP*WP] (two-level solve)
    const cplx<T>* Fa;    // complex64: G_l in phase-A operand order, [Ny][WP*WP] (see helm_internal.hpp)
    const cplx<T>* Fw;    // complex64: chain blocks in operand order, [P-1][4][WP*WP]
    cplx<T>* Yw;          // workspace [nrhs][Ny][WP]
    const double2* cy;
    const double2* by;
    IOSpec io;
    int Ny, W, m, P, nrhs;
    int q, G;             // separator groups (two-level separator solve when G >= 2)
};

// Block coordinates of a workgroup: the launch's own (one problem), or its place inside one
// problem of a multi-problem launch (nz: the number of z blocks that problem uses).
struct Blk {
    int x, y, z, nz;
};
__device__ inline Blk own_blk() { return Blk{(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z, (int)gridDim.z}; }

// Several problems' strip solves in one launch (one strip of each): their arguments by value
// in the kernel-argument block, x blocks [xs[k], xs[k+1]) belonging to problem k, which uses
// ny[k] y blocks and nz[k] z blocks of the launch's maximum (the others return at once).
template <typename T>
struct MultiArgs {
    SolveArgs<T> a[MULTI_MAX];
    int xs[MULTI_MAX + 1];
    int ny[MULTI_MAX], nz[MULTI_MAX];
    int n;
};
static_assert(sizeof(MultiArgs<float>) <= 4096, "multi-problem arguments exceed the kernel-argument block");

// problem of this workgroup and its block coordinates inside it; false: idle workgroup
template <typename T>
__device__ inline bool multi_blk(const MultiArgs<T>& m, int& k, Blk& b) {
    const int bx = (int)blockIdx.x;
    k = 0;
    while (k + 1 < m.n && bx >= m.xs[k + 1]) ++k;
    b = Blk{bx - m.xs[k], (int)blockIdx.y, (int)blockIdx.z, m.nz[k]};
    return b.y < m.ny[k] && b.z < m.nz[k];
}

template <typename T>
__device__ inline cplx<T> gather(const IOSpec& io, int r, int l, int q, int Ny) {
    double2 v = cmk<double2>(0.0, 0.0);
    if (q >= io.src_lo && q < io.src_hi)
        v = io.src[(size_t)r * io.src_rs + (size_t)l * io.src_ls + (q + io.src_off)];
    if (tr_col(io, q)) {
        const double2 ta = io.trA[(size_t)r * Ny + l], tb = io.trB[(size_t)r * Ny + l];
        v.x += io.coef * (tb.x - ta.x);
        v.y += io.coef * (tb.y - ta.y);
    }
    return ccast<cplx<T>>(v);
}

// Branch-free gather in two halves: load_raw issues the loads (clamped addresses; lanes
// outside the source or transmission columns read element 0 and discard it), combine
// forms the right-hand-side value.  Keeping the uses apart from the loads lets the loads
// of the next step overlap the current one.  io.src, io.trA and io.trB must be valid
// pointers (the host points unused transmission traces at the source).
struct RawRhs {
    double2 v, ta, tb;
};
__device__ inline RawRhs load_raw(const IOSpec& io, int r, int l, int q, int Ny, int nrhs, int W) {
    const bool ok = r < nrhs && q < W;
    const bool in_src = ok && q >= io.src_lo && q < io.src_hi;
    const bool in_tr = ok && tr_col(io, q);
    const size_t ps = in_src ? (size_t)r * io.src_rs + (size_t)l * io.src_ls + (q + io.src_off) : 0;
    const size_t pt = in_tr ? (size_t)r * Ny + l : 0;
    RawRhs x;
    x.v = io.src[ps];
    x.ta = io.trA[pt];
    x.tb = io.trB[pt];
    if (!in_src) x.v = cmk<double2>(0.0, 0.0);
    if (!in_tr) { x.ta = cmk<double2>(0.0, 0.0); x.tb = x.ta; }
    return x;
}
// The same for the four consecutive columns q0 .. q0 + 3 of one row: the transmission term
// is the same for both of its columns, so the two trace values are loaded once.
struct RawRhs4 {
    double2 v[4];
    double2 ta, tb;
};
__device__ inline void load_raw4(RawRhs4& x, const IOSpec& io, int r, int l, int q0, int Ny, int nrhs, int W) {
    const bool rok = r < nrhs;
    const bool tr = rok && io.q_t >= 0 && io.q_t + 1 >= q0 && io.q_t <= q0 + 3;
    const size_t pt = tr ? (size_t)r * Ny + l : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int q = q0 + j;
        const bool in_src = rok && q < W && q >= io.src_lo && q < io.src_hi;
        const size_t ps = in_src ? (size_t)r * io.src_rs + (size_t)l * io.src_ls + (q + io.src_off) : 0;
        x.v[j] = io.src[ps];
        if (!in_src) x.v[j] = cmk<double2>(0.0, 0.0);
    }
    x.ta = io.trA[pt];
    x.tb = io.trB[pt];
    if (!tr) { x.ta = cmk<double2>(0.0, 0.0); x.tb = x.ta; }
}
__device__ inline float2 combine4(const IOSpec& io, const RawRhs4& x, int j, int q) {
    double2 v = x.v[j];
    if (tr_col(io, q)) {
        v.x += io.coef * (x.tb.x - x.ta.x);
        v.y += io.coef * (x.tb.y - x.ta.y);
    }
    return make_float2((float)v.x, (float)v.y);
}

template <typename T>
__device__ inline cplx<T> combine(const IOSpec& io, const RawRhs& x) {
    double2 v = x.v;
    v.x += io.coef * (x.tb.x - x.ta.x);
    v.y += io.coef * (x.tb.y - x.ta.y);
    return ccast<cplx<T>>(v);
}

template <typename T>
__device__ inline const cplx<T>* fslot(const SolveArgs<T>& a, int l, int sl) {
    return a.F + ((size_t)l * NSLOT + sl) * BLK;
}

template <typename T>
__device__ inline void scatter(const SolveArgs<T>& a, int r, int l, int i, cplx<T> x) {
    const IOSpec& io = a.io;
    const double2 xv = ccast<double2>(x);
    const bool o0 = i >= io.o_lo[0] && i < io.o_hi[0];
    const bool o = o0 || (i >= io.o_lo[1] && i < io.o_hi[1]);
    if (o && io.dst) {
        double2* p = io.dst + (size_t)r * io.dst_rs + (size_t)l * io.dst_ls + (i + io.dst_off[o0 ? 0 : 1]);
        *p = io.accumulate ? cadd(*p, xv) : xv;
    }
    if (i == io.qo0 && io.tro0) io.tro0[(size_t)r * a.Ny + l] = xv;
    if (i == io.qo1 && io.tro1) io.tro1[(size_t)r * a.Ny + l] = xv;
}

// A factor block staged through registers into LDS.  Thread t owns elements
// t + NT*j, j < BLK/NT, of the column-major block.
template <typename T>
struct BlockPipe {
    static constexpr int PER = BLK / NT;
    cplx<T> reg[PER];
    __device__ void load(const cplx<T>* __restrict__ g) {
#pragma unroll
        for (int j = 0; j < PER; ++j) reg[j] = g[threadIdx.x + NT * j];
    }
    __device__ void store(cplx<T>* s) const {
#pragma unroll
        for (int j = 0; j < PER; ++j) s[threadIdx.x + NT * j] = reg[j];
    }
};

// acc[u] += sum_{k<W} M(i,k) vin[k][g + G*u]   (M column-major WP x WP)
template <typename T, int R, int G>
__device__ inline void matvec(cplx<T> (&acc)[R / G], const cplx<T>* M, const cplx<T> (*vin)[R],
                              int W, int i, int g) {
    constexpr int U = R / G;
#pragma unroll 4
    for (int k = 0; k < W; ++k) {
        const cplx<T> mk = M[k * WP + i];
#pragma unroll
        for (int u = 0; u < U; ++u) cfma(acc[u], mk, vin[k][g + G * u]);
    }
}

// ---------------------------------------------------------------- phase A
// R right-hand sides per workgroup; thread (i = t % 64, g = t / 64) owns row i of the
// block and right-hand sides g, g+4, ...
template <typename T, int R>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 1))) k_phase_a(SolveArgs<T> a) {
    using V = cplx<T>;
    constexpr int G = 4, U = R / G;
    __shared__ V Gs[2][BLK];
    __shared__ V vin[WP][R];
    const int t = threadIdx.x, i = t & (WP - 1), g = t >> 6;
    const int c = blockIdx.x, rbase = blockIdx.y * R;
    const int r0 = c * a.m;
    const int r1 = (c < a.P - 1) ? c * a.m + a.m - 1 : a.Ny;
    const int n = r1 - r0;
    const int steps = 2 * n - 1;                 // forward r0..r1-1, backward r1-2..r0
    auto row_of = [&](int k) { return k < n ? r0 + k : r1 - 2 - (k - n); };
    const V zero = cmk<V>(0, 0);
    V z[U];
#pragma unroll
    for (int u = 0; u < U; ++u) z[u] = zero;

    // the next step's block, staged through registers as separate real and imaginary parts
    // (an array of complex128 values was kept in scratch memory)
    constexpr int PER = BLK / NT;
    T prx[PER], pry[PER];
    auto pload = [&](const V* __restrict__ gsrc) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const V v = gsrc[t + NT * j];
            prx[j] = v.x;
            pry[j] = v.y;
        }
    };
    auto pstore = [&](V* dst) {
#pragma unroll
        for (int j = 0; j < PER; ++j) dst[t + NT * j] = cmk<V>(prx[j], pry[j]);
    };
    pload(fslot(a, row_of(0), 0));
    pstore(Gs[0]);
    int cur = 0;
    for (int k = 0; k < steps; ++k) {
        const int l = row_of(k);
        const bool fwd = k < n;
        // unconditional (the last step reloads its own block)
        pload(fslot(a, row_of(k + 1 < steps ? k + 1 : k), 0));
        if (fwd) {
            const V cl = ccast<V>(a.cy[l]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int r = rbase + g + G * u;
                V v = zero;
                if (r < a.nrhs && i < a.W) {
                    v = gather<T>(a.io, r, l, i, a.Ny);
                    if (l > r0) v = csub(v, cmul(cl, z[u]));
                }
                vin[i][g + G * u] = v;
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) vin[i][g + G * u] = z[u];
        }
        __syncthreads();
        V acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = zero;
        matvec<T, R, G>(acc, Gs[cur], vin, a.W, i, g);
        if (fwd) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int r = rbase + g + G * u;
                z[u] = acc[u];
                if (r < a.nrhs) a.Yw[((size_t)r * a.Ny + l) * WP + i] = acc[u];
            }
        } else {
            const V bl = ccast<V>(a.by[l]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int r = rbase + g + G * u;
                if (r < a.nrhs) {
                    V* p = a.Yw + ((size_t)r * a.Ny + l) * WP + i;
                    const V y = csub(*p, cmul(bl, acc[u]));
                    *p = y;
                    z[u] = y;
                } else {
                    z[u] = zero;
                }
            }
        }
        pstore(Gs[cur ^ 1]);
        __syncthreads();
        cur ^= 1;
    }
}

// ---------------------------------------------------------------- phase A, MFMA
// complex64, 16 right-hand sides per workgroup.  The block product Z = G V (64 x 64 times
// 64 x 16, complex) runs on v_mfma_f32_16x16x4f32 as three real products (Gauss's form:
// M1 = Gr Vr, M2 = Gi Vi, M3 = (Gr + Gi)(Vr + Vi), Zr = M1 - M2, Zi = M3 - M1 - M2; 48
// instead of 64 MFMAs per step, 126 instead of 133 us per launch at 2000^2, iteration
// counts unchanged); wave w owns output rows 16w..16w+15.
// MFMA lane layout (16x16x4, one block): A[l % 16][l / 16], B[l / 16][l % 16],
// C[4 (l / 16) + j][l % 16] in component j.
typedef float mf4 __attribute__((ext_vector_type(4)));

// The blocks G_l are not staged through LDS: each lane loads exactly its MFMA A operands
// (16 values per block, A[16w + n][4s + q4] for k-step s) straight from global memory into
// a ring of D register blocks, D steps ahead.  Only the right-hand-side panel of a step
// (64 x 16) goes through LDS, double-buffered, so a step has a single barrier.  Each lane
// gathers the right-hand-side values of its own four output positions.  The ring slot a
// step's products read is refilled inside the product loop, one 16-byte load after the six
// products that read its pair: the four waves of a workgroup reach their products together
// after the barrier, and loads issued after the products kept the CU's load path busy
// while the matrix cores idled (and the stores and right-hand-side loads queued behind).
template <int D>
__device__ __forceinline__ void phase_a_mfma(const SolveArgs<float>& a, const Blk& B) {
    using V = float2;
    constexpr int R = 16;
    __shared__ V Vs[2][WP][R];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int n = lane & 15, q4 = lane >> 4;            // MFMA column (rhs), row quad
    const int c = B.x, rbase = B.y * R;
    const int r0 = c * a.m;
    const int r1 = (c < a.P - 1) ? c * a.m + a.m - 1 : a.Ny;
    const int nr = r1 - r0;
    const int nsteps = 2 * nr - 1;                       // forward nr rows, backward nr - 1
    const V zero = make_float2(0.f, 0.f);
    const int rn = rbase + n;                            // rhs of this lane's MFMA column
    const bool rn_ok = rn < a.nrhs;
    const int qrow = 16 * w + 4 * q4;                    // first of this lane's 4 output rows
    const size_t ybase = (size_t)(rn_ok ? rn : 0) * a.Ny * WP + qrow;
    // targets-only solves read y at the compact target columns (phase C) and on the first
    // and last interior row (the separators' right-hand sides); full solves read it all
    bool tm[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        bool on = false;
        for (int k = 0; k < 8; ++k) on = on || (a.tcol[k] == qrow + j);
        tm[j] = on;
    }
    auto row_of = [&](int k) {
        k = k < nsteps ? k : nsteps - 1;
        return k < nr ? r0 + k : r1 - 2 - (k - nr);
    };
    // the A operands of k-steps 2i and 2i + 1 come in one 16-byte load (operand-order copy)
    auto g_ptr = [&](int k) {
        return reinterpret_cast<const float4*>(a.Fa + (size_t)row_of(k) * BLK) + w * 8 * 64 + lane;
    };
    auto load_g = [&](int k, V (&g)[16]) {
        const float4* G = g_ptr(k);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float4 v = G[i * 64];
            g[2 * i] = make_float2(v.x, v.y);
            g[2 * i + 1] = make_float2(v.z, v.w);
        }
    };
    RawRhs4 raw;
    auto load_rhs = [&](int l) {
        load_raw4(raw, a.io, rn, l, qrow, a.Ny, a.nrhs, a.W);
    };
    V greg[D][16];
    V z[4], zn[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) { z[j] = zero; zn[j] = zero; }
    double2 cnext = a.cy[r0], bnext = a.by[r0];
    load_rhs(r0);
#pragma unroll
    for (int d = 0; d < D; ++d) load_g(d, greg[d]);

    // products of block g with the staged panel; g is refilled with block knext meanwhile
    auto mfma_block = [&](V (&g)[16], const V (*Vb)[R], V (&out)[4], int knext) {
        const float4* Gn = g_ptr(knext);
        // three real products per complex one: M1 = Gr Vr, M2 = Gi Vi, M3 = (Gr + Gi)(Vr + Vi);
        // Zr = M1 - M2, Zi = M3 - M1 - M2
        mf4 m1 = {0.f, 0.f, 0.f, 0.f}, m2 = m1, m3 = m1, n1 = m1, n2 = m1, n3 = m1;
        V vb[16];
#pragma unroll
        for (int s4 = 0; s4 < 16; ++s4) vb[s4] = Vb[4 * s4 + q4][n];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s4 = 0; s4 < 16; s4 += 2) {
            const V g0 = g[s4], g1 = g[s4 + 1];
            const V v0 = vb[s4], v1 = vb[s4 + 1];
            m1 = __builtin_amdgcn_mfma_f32_16x16x4f32(g0.x, v0.x, m1, 0, 0, 0);
            m2 = __builtin_amdgcn_mfma_f32_16x16x4f32(g0.y, v0.y, m2, 0, 0, 0);
            m3 = __builtin_amdgcn_mfma_f32_16x16x4f32(g0.x + g0.y, v0.x + v0.y, m3, 0, 0, 0);
            n1 = __builtin_amdgcn_mfma_f32_16x16x4f32(g1.x, v1.x, n1, 0, 0, 0);
            n2 = __builtin_amdgcn_mfma_f32_16x16x4f32(g1.y, v1.y, n2, 0, 0, 0);
            n3 = __builtin_amdgcn_mfma_f32_16x16x4f32(g1.x + g1.y, v1.x + v1.y, n3, 0, 0, 0);
            const float4 nv = Gn[(s4 >> 1) * 64];
            g[s4] = make_float2(nv.x, nv.y);
            g[s4 + 1] = make_float2(nv.z, nv.w);
            __builtin_amdgcn_sched_group_barrier(0x008, 6, 0);   // six MFMAs,
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // then the pair's load
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float p1 = m1[j] + n1[j], p2 = m2[j] + n2[j], p3 = m3[j] + n3[j];
            out[j] = make_float2(p1 - p2, p3 - p1 - p2);
        }
    };

    // component-wise select (a select of whole float2 values goes through scratch memory)
    auto keep = [](bool on, V x) { return make_float2(on ? x.x : 0.f, on ? x.y : 0.f); };
    // ---- forward row l = r0 + k:  z_l = G_l (r_l - c_l z_{l-1})
    auto fwd_step = [&](int k, int j) {
        const int buf = k & 1;
        const int l = r0 + k;
        // the first row of a chunk has no coupling inside phase A (scalar selects: no
        // aggregate select that would go through memory)
        const float clx = k > 0 ? (float)cnext.x : 0.f, cly = k > 0 ? (float)cnext.y : 0.f;
        const V cl = make_float2(clx, cly);
        V v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = csub(combine4(a.io, raw, u, qrow + u), cmul(cl, z[u]));
        // next step's small loads first (vmcnt retires in issue order); clamped, branch-free
        const int ln = l + 1 < r1 ? l + 1 : l;
        cnext = a.cy[ln];
        load_rhs(ln);
#pragma unroll
        for (int u = 0; u < 4; ++u) Vs[buf][qrow + u][n] = v[u];
        __syncthreads();
        V acc[4];
        mfma_block(greg[j], Vs[buf], acc, k + D);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            z[u] = keep(rn_ok, acc[u]);
            if (rn_ok) a.Yw[ybase + (size_t)l * WP + u] = acc[u];
        }
    };
    // ---- backward row l = r1 - 2 - (k - nr):  y_l = z_l - b_l G_l y_{l+1}
    auto bwd_step = [&](int k, int j) {
        const int buf = k & 1;
        const int l = r1 - 2 - (k - nr);
        V zl[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) zl[u] = zn[u];
        const V bl = ccast<V>(bnext);
        const int lb = l - 1 >= r0 ? l - 1 : l;
        bnext = a.by[lb];
#pragma unroll
        for (int u = 0; u < 4; ++u) zn[u] = a.Yw[ybase + (size_t)lb * WP + u];
#pragma unroll
        for (int u = 0; u < 4; ++u) Vs[buf][qrow + u][n] = z[u];
        __syncthreads();
        V acc[4];
        mfma_block(greg[j], Vs[buf], acc, k + D);
        const bool store_y = !a.io.targets_only || l == r0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const V y = csub(zl[u], cmul(bl, acc[u]));
            z[u] = keep(rn_ok, y);
            if (rn_ok && (store_y || tm[u])) a.Yw[ybase + (size_t)l * WP + u] = y;
        }
    };
    int k = 0;
    for (; k + D <= nr; k += D) {
#pragma unroll
        for (int j = 0; j < D; ++j) fwd_step(k + j, j);
    }
#pragma unroll
    for (int j = 0; j < D; ++j)
        if (k + j < nr) fwd_step(k + j, j);
    if (nr < 2) return;
    // z_{r1-2} and b_{r1-2} of the first backward row (ybase is valid for every lane: lanes
    // beyond nrhs read rows of right-hand side 0 and discard them)
    bnext = a.by[r1 - 2];
#pragma unroll
    for (int u = 0; u < 4; ++u) zn[u] = a.Yw[ybase + (size_t)(r1 - 2) * WP + u];
    // backward steps k = nr .. 2 nr - 2 use ring slot k % D: the loop is unrolled for the
    // slot of its first step
    auto bwd_loop = [&](auto off_tag) {
        constexpr int OFF = decltype(off_tag)::value;
        int kb = nr;
        for (; kb + D <= nsteps; kb += D) {
#pragma unroll
            for (int j = 0; j < D; ++j) bwd_step(kb + j, (j + OFF) % D);
        }
#pragma unroll
        for (int j = 0; j < D; ++j)
            if (kb + j < nsteps) bwd_step(kb + j, (j + OFF) % D);
    };
    static_assert(D >= 1 && D <= 4, "ring alignment dispatch below covers D <= 4");
    const int off = nr % D;
    if (off == 0) bwd_loop(std::integral_constant<int, 0>{});
    if constexpr (D > 1) { if (off == 1) bwd_loop(std::integral_constant<int, 1 % D>{}); }
    if constexpr (D > 2) { if (off == 2) bwd_loop(std::integral_constant<int, 2 % D>{}); }
    if constexpr (D > 3) { if (off == 3) bwd_loop(std::integral_constant<int, 3 % D>{}); }
}
template <int D>
__global__ void __launch_bounds__(NT) k_phase_a_mfma(SolveArgs<float> a) { phase_a_mfma<D>(a, own_blk()); }
template <int D>
__global__ void __launch_bounds__(NT) k_phase_a_mfma_multi(MultiArgs<float> m) {
    int k;
    Blk b;
    if (multi_blk(m, k, b)) phase_a_mfma<D>(m.a[k], b);
}

// ---------------------------------------------------------------- phase B0
// a_c = G'_c r^_c for every separator (grid: separators x rhs groups), stored at row s_c.
template <typename T, int R>
__global__ void __launch_bounds__(NT) k_phase_b0(SolveArgs<T> a) {
    using V = cplx<T>;
    constexpr int G = 4, U = R / G;
    __shared__ V vin[WP][R];
    const int t = threadIdx.x, i = t & (WP - 1), g = t >> 6;
    const int c = blockIdx.x, rbase = blockIdx.y * R;
    const int s = c * a.m + a.m - 1;
    const V cs = ccast<V>(a.cy[s]), bs = ccast<V>(a.by[s]);
    const V zero = cmk<V>(0, 0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int r = rbase + g + G * u;
        V v = zero;
        if (r < a.nrhs && i < a.W) {
            v = gather<T>(a.io, r, s, i, a.Ny);
            v = csub(v, cmul(cs, a.Yw[((size_t)r * a.Ny + (s - 1)) * WP + i]));
            v = csub(v, cmul(bs, a.Yw[((size_t)r * a.Ny + (s + 1)) * WP + i]));
        }
        vin[i][g + G * u] = v;
    }
    __syncthreads();
    V acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = zero;
    matvec<T, R, G>(acc, fslot(a, s, 0), vin, a.W, i, g);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int r = rbase + g + G * u;
        if (r < a.nrhs) a.Yw[((size_t)r * a.Ny + s) * WP + i] = acc[u];
    }
}

// ---------------------------------------------------------------- phase B
// One right-hand side per workgroup; the k-sum of every matvec is split over the 4 waves
// and combined through LDS.  Forward z'_0 = a_0, z'_c = a_c - K_c z'_{c-1}; backward
// x_{P-2} = z'_{P-2}, x_c = z'_c - U'_c x_{c+1}.  The blocks of the next D steps are in
// flight in registers while a step runs (ring of D+1 LDS buffers).
constexpr int ZMAX = 64;   // separators whose z' the chain keeps in LDS

// Thread (i, w) owns row i of the matvec and the 16 columns 16w..16w+15 of every block:
// the blocks of the next D steps are loaded straight into registers in that layout (no
// LDS staging), so a step is 16 multiply-adds from registers, one partial-sum exchange
// and two barriers.  ZB: the forward results z'_c stay in LDS (zb) for the backward pass
// and the forward inputs a_c are loaded D steps ahead into a register ring (requires
// P - 1 <= ZMAX); otherwise the next input is loaded one step ahead from global memory.
template <typename T, int D, bool ZB>
__global__ void __launch_bounds__(NT) k_phase_b(SolveArgs<T> a) {
    using V = cplx<T>;
    __shared__ V vec[WP];
    __shared__ V part[4][WP];
    __shared__ V zb[ZB ? ZMAX + 1 : 1][WP];     // row ZMAX: discard row for backward steps
    const int t = threadIdx.x, i = t & (WP - 1), w = t >> 6;
    const int r = blockIdx.x;
    const int ns = a.P - 1;                  // separators
    const int nf = ns - 1;                   // forward steps (c = 1..ns-1)
    const int steps = nf + (ns - 1);         // + backward steps (c = ns-2..0)
    if (steps <= 0) return;
    const int k0 = w * 16;
    auto sep = [&](int c) { return c * a.m + a.m - 1; };
    // separator row and factor block of step k (clamped to the last step: loads past the
    // end re-read the last block and are never used)
    auto sep_of = [&](int k) {
        k = k < steps ? k : steps - 1;
        return sep(k < nf ? k + 1 : ns - 2 - (k - nf));
    };
    auto blk = [&](int k) {
        k = k < steps ? k : steps - 1;
        return k < nf ? fslot(a, sep(k + 1), 1) : fslot(a, sep(ns - 2 - (k - nf)), 2);
    };
    auto load_blk = [&](int k, V (&b)[16]) {
        const V* g = blk(k) + (size_t)k0 * WP + i;
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) b[kk] = g[kk * WP];
    };
    // forward input of step k: a_{k+1} (clamped to the last forward step)
    auto fwd_in = [&](int k) { return sep((k < nf ? k : nf - 1) + 1); };
    V* Yr = a.Yw + (size_t)r * a.Ny * WP;
    // every thread keeps the value of its row i; the four waves hold identical copies
    const V a0 = Yr[(size_t)sep(0) * WP + i];    // z'_0 = a_0
    vec[i] = a0;
    V nextv = cmk<V>(0, 0);
    V av[D];
    if (ZB) {
        zb[0][i] = a0;
#pragma unroll
        for (int d = 0; d < D; ++d) av[d] = Yr[(size_t)fwd_in(d) * WP + i];
    } else {
        nextv = Yr[(size_t)sep_of(0) * WP + i];
    }
    V breg[D][16];
#pragma unroll
    for (int d = 0; d < D; ++d) load_blk(d, breg[d]);
    __syncthreads();
    auto step = [&](int k, int j) {
        const int s = sep_of(k);
        const bool fwd = k < nf;
        V curv;                                  // a_c (forward) or z'_c (backward)
        if (ZB) {
            const int cb = fwd ? ZMAX : ns - 2 - (k - nf);
            const V zr = zb[cb][i];
            curv = fwd ? av[j] : zr;
            av[j] = Yr[(size_t)fwd_in(k + D) * WP + i];
        } else {
            curv = nextv;
            nextv = Yr[(size_t)sep_of(k + 1) * WP + i];
        }
        V acc0 = cmk<V>(0, 0), acc1 = acc0;
#pragma unroll
        for (int kk = 0; kk < 16; kk += 2) {
            cfma(acc0, breg[j][kk], vec[k0 + kk]);
            cfma(acc1, breg[j][kk + 1], vec[k0 + kk + 1]);
        }
        part[w][i] = cadd(acc0, acc1);
        load_blk(k + D, breg[j]);               // block of step k + D into the freed slot
        __syncthreads();
        const V sum = cadd(cadd(part[0][i], part[1][i]), cadd(part[2][i], part[3][i]));
        const V v = csub(curv, sum);            // a_c - K_c z'  or  z'_c - U'_c x
        Yr[(size_t)s * WP + i] = v;
        vec[i] = v;
        if (ZB) zb[fwd ? k + 1 : ZMAX][i] = v;
        __syncthreads();
    };
    int k = 0;
    for (; k + D <= steps; k += D) {
#pragma unroll
        for (int j = 0; j < D; ++j) step(k + j, j);
    }
#pragma unroll
    for (int j = 0; j < D; ++j)
        if (k + j < steps) step(k + j, j);
}

// ---------------------------------------------------------------- phase B, two levels
// The separator recurrences are cut into G groups of q separators.  With zeta / xi the
// recurrences of a group started from zero and the propagators Phi / Psi of the factor,
//   forward   z'_c = zeta_c + Phi_c z'_{first-1},   backward  x_c = xi_c + Psi_c x_{last+1},
// so the solve is: local forward chains (all groups in parallel), a chain over the groups'
// last separators, fix-up + local backward chains (parallel), a chain over the groups'
// first separators, fix-up (parallel): about 2q + 2G dependent steps instead of 2(P-1).
// A workgroup takes RB right-hand sides (every block it loads serves all of them); entries
// of right-hand sides beyond nrhs (a ragged last group) are computed from clamped loads and
// never stored.  The chains are latency bound: at 64 right-hand sides one per workgroup was
// the fastest (separator solve per strip 77 us; two per workgroup 84, four 105, eight 237).
//
// sep_chain: thread (i, w) owns row i and the 16 columns 16w..16w+15 of every block; wave
// w keeps its own copy of the vectors (their 16 entries it reads are produced by its own
// lanes), so a step needs one barrier (for the 4-wave partial sums).  Step k:
//   v_k = in_k + sgn (M_k vec),  out_k = v_k,  vec = v_k if chain (else vec stays v0).
// Blocks and inputs of the next D steps are in flight in registers.
template <typename T> struct SepRB { static constexpr int RB = 1; };

// SW: blk(k) is an operand-order block of Fw (complex64): the lane's columns 16 w + 2 j,
// 16 w + 2 j + 1 come in one 16-byte load; otherwise a factor block in its own layout.
template <typename T, int D, int RB, bool SW = false, typename BF, typename RF>
__device__ void sep_chain(int n, bool chain, const cplx<T> (&v0)[RB], T sgn, BF blk, RF row,
                          const bool (&okb)[RB], cplx<T> (*vecw)[RB][WP], cplx<T> (*part)[4][RB][WP]) {
    using V = cplx<T>;
    if (n <= 0) return;
    const int t = threadIdx.x, i = t & (WP - 1), w = t >> 6, k0 = 16 * w;
#pragma unroll
    for (int b = 0; b < RB; ++b) vecw[w][b][i] = v0[b];
    __builtin_amdgcn_wave_barrier();   // the wave's own lanes produced the entries it reads
    V breg[D][16], ireg[D][RB];
    auto load = [&](int k, V (&bl)[16], V (&x)[RB]) {
        const int kc = k < n ? k : n - 1;
        if constexpr (SW) {
            const float4* M = reinterpret_cast<const float4*>(blk(kc)) + w * 8 * 64 + i;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float4 v = M[j * 64];
                bl[2 * j] = make_float2(v.x, v.y);
                bl[2 * j + 1] = make_float2(v.z, v.w);
            }
        } else {
            const V* M = blk(kc) + (size_t)k0 * WP + i;
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) bl[kk] = M[kk * WP];
        }
#pragma unroll
        for (int b = 0; b < RB; ++b) x[b] = row(kc, b)[i];
    };
#pragma unroll
    for (int d = 0; d < D; ++d) load(d, breg[d], ireg[d]);
    auto step = [&](int k, int j) {
        V acc[RB];
#pragma unroll
        for (int b = 0; b < RB; ++b) acc[b] = cmk<V>(0, 0);
#pragma unroll
        for (int kk = 0; kk < 16; ++kk)
#pragma unroll
            for (int b = 0; b < RB; ++b) cfma(acc[b], breg[j][kk], vecw[w][b][k0 + kk]);
        V xin[RB];
#pragma unroll
        for (int b = 0; b < RB; ++b) xin[b] = ireg[j][b];
        load(k + D, breg[j], ireg[j]);
#pragma unroll
        for (int b = 0; b < RB; ++b) part[k & 1][w][b][i] = acc[b];
        __syncthreads();
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const V sum = cadd(cadd(part[k & 1][0][b][i], part[k & 1][1][b][i]),
                               cadd(part[k & 1][2][b][i], part[k & 1][3][b][i]));
            const V v = cmk<V>(xin[b].x + sgn * sum.x, xin[b].y + sgn * sum.y);
            if (okb[b]) row(k, b)[i] = v;
            if (chain) vecw[w][b][i] = v;
        }
        __builtin_amdgcn_wave_barrier();
    };
    int k = 0;
    for (; k + D <= n; k += D) {
#pragma unroll
        for (int j = 0; j < D; ++j) step(k + j, j);
    }
#pragma unroll
    for (int j = 0; j < D; ++j)
        if (k + j < n) step(k + j, j);
    __syncthreads();
}

// Independent updates v_k = in_k + M_k v (k < n, the same vectors v for every k): wave w
// takes k = w, w + 4, ..., each lane one row of the full 64-column products, so the waves
// need no barrier between updates.  v0 holds this lane's entries of the vectors.
template <typename T, int RB, typename BF, typename RF>
__device__ void sep_fix(int n, const cplx<T> (&v0)[RB], BF blk, RF row, const bool (&okb)[RB],
                        cplx<T> (*vecw)[RB][WP]) {
    using V = cplx<T>;
    const int i = threadIdx.x & (WP - 1), w = threadIdx.x >> 6;
#pragma unroll
    for (int b = 0; b < RB; ++b) vecw[w][b][i] = v0[b];
    __builtin_amdgcn_wave_barrier();
    for (int k = w; k < n; k += 4) {
        const V* M = blk(k) + i;
        V acc[RB];
#pragma unroll
        for (int b = 0; b < RB; ++b) acc[b] = cmk<V>(0, 0);
#pragma unroll 16
        for (int kk = 0; kk < WP; ++kk) {
            const V m = M[(size_t)kk * WP];
#pragma unroll
            for (int b = 0; b < RB; ++b) cfma(acc[b], m, vecw[w][b][kk]);
        }
#pragma unroll
        for (int b = 0; b < RB; ++b)
            if (okb[b]) {
                V* dst = row(k, b) + i;
                *dst = cadd(*dst, acc[b]);
            }
    }
    __syncthreads();
}

template <typename T>
struct SepCtx {
    const SolveArgs<T>& a;
    int ns, rbase;
    __device__ int sep(int c) const { return c * a.m + a.m - 1; }
    __device__ int first(int g) const { return g * a.q; }
    __device__ int last(int g) const { return min(g * a.q + a.q, ns) - 1; }
    __device__ const cplx<T>* prop(int c, int dir) const { return a.Fs + ((size_t)c * 2 + dir) * BLK; }
    __device__ bool ok(int b) const { return rbase + b < a.nrhs; }
    __device__ int rhs(int b) const { return rbase + b < a.nrhs ? rbase + b : a.nrhs - 1; }   // clamped
    __device__ cplx<T>* yrow(int b, int c) const { return a.Yw + ((size_t)rhs(b) * a.Ny + sep(c)) * WP; }
};

#define SEPK_PROLOGUE_N(RBN)                                              \
    using V = cplx<T>;                                                    \
    constexpr int RB = (RBN);                                             \
    __shared__ V vecw[4][RB][WP];                                         \
    __shared__ V part[2][4][RB][WP];                                      \
    const int i = threadIdx.x & (WP - 1);                                 \
    SepCtx<T> X{a, a.P - 1, B.x * RB};                                    \
    bool okb[RB];                                                         \
    for (int b = 0; b < RB; ++b) okb[b] = X.ok(b);                        \
    auto vecs_at = [&](int c, V (&v)[RB]) {                               \
        for (int b = 0; b < RB; ++b) v[b] = X.yrow(b, c)[i];              \
    };                                                                    \
    (void)i;
#define SEPK_PROLOGUE SEPK_PROLOGUE_N(SepRB<T>::RB)
// The local chains without their independent products run 8 groups x the right-hand sides
// as workgroups: two right-hand sides per workgroup (every block load serves both) keep
// one workgroup per CU, which measured faster than two workgroups of one.
template <typename T> struct SepLocalRB { static constexpr int RB = 2; };

// local forward chains: zeta_c = a_c - K_c zeta_{c-1} inside group g = blockIdx.y.  First
// the group's right-hand sides a_c = G'_c r^_c, r^_c = r_s - c_s y_{s-1} - b_s y_{s+1}
// (s = sep(c)), independent per separator: wave w takes c0 + w, c0 + w + 4, ...
template <typename T, int D, bool SETUP>
__device__ __forceinline__ void sep_fwd_local(const SolveArgs<T>& a, const Blk& B) {
    SEPK_PROLOGUE_N(SETUP ? SepRB<T>::RB : SepLocalRB<T>::RB)
    const int g = B.y, c0 = X.first(g), c1 = X.last(g);
    if constexpr (SETUP) {
        const int w = threadIdx.x >> 6;
        for (int c = c0 + w; c <= c1; c += 4) {
            const int sr = X.sep(c);
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                const int r = X.rhs(b);
                const V* Yr = a.Yw + (size_t)r * a.Ny * WP;
                V v = cmk<V>(0, 0);
                if (i < a.W) {
                    v = gather<T>(a.io, r, sr, i, a.Ny);
                    v = csub(v, cmul(ccast<V>(a.cy[sr]), Yr[(size_t)(sr - 1) * WP + i]));
                    v = csub(v, cmul(ccast<V>(a.by[sr]), Yr[(size_t)(sr + 1) * WP + i]));
                }
                vecw[w][b][i] = v;
            }
            __builtin_amdgcn_wave_barrier();
            const V* M = fslot(a, sr, 0) + i;
            V acc[RB];
#pragma unroll
            for (int b = 0; b < RB; ++b) acc[b] = cmk<V>(0, 0);
#pragma unroll 16
            for (int kk = 0; kk < WP; ++kk) {
                const V m = M[(size_t)kk * WP];
#pragma unroll
                for (int b = 0; b < RB; ++b) cfma(acc[b], m, vecw[w][b][kk]);
            }
#pragma unroll
            for (int b = 0; b < RB; ++b)
                if (okb[b]) a.Yw[((size_t)X.rhs(b) * a.Ny + sr) * WP + i] = acc[b];
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
    }
    V v0[RB];
    vecs_at(c0, v0);
    if constexpr (!SETUP && std::is_same<T, float>::value)
        sep_chain<T, D, RB, true>(c1 - c0, true, v0, T(-1),
                                  [&](int k) { return a.Fw + ((size_t)(c0 + 1 + k) * 4 + 0) * BLK; },
                                  [&](int k, int b) { return X.yrow(b, c0 + 1 + k); }, okb, vecw, part);
    else
        sep_chain<T, D, RB>(c1 - c0, true, v0, T(-1),
                            [&](int k) { return fslot(a, X.sep(c0 + 1 + k), 1); },
                            [&](int k, int b) { return X.yrow(b, c0 + 1 + k); }, okb, vecw, part);
}

// chain over the groups' last separators: z'_{last g} = zeta_{last g} + Phi_{last g} z'_{last g-1}
template <typename T, int D>
__device__ __forceinline__ void sep_fwd_top(const SolveArgs<T>& a, const Blk& B) {
    SEPK_PROLOGUE
    V v0[RB];
    vecs_at(X.last(0), v0);
    if constexpr (std::is_same<T, float>::value)
        sep_chain<T, D, RB, true>(a.G - 1, true, v0, T(1),
                                  [&](int k) { return a.Fw + ((size_t)X.last(k + 1) * 4 + 2) * BLK; },
                                  [&](int k, int b) { return X.yrow(b, X.last(k + 1)); }, okb, vecw, part);
    else
        sep_chain<T, D, RB>(a.G - 1, true, v0, T(1),
                            [&](int k) { return X.prop(X.last(k + 1), 0); },
                            [&](int k, int b) { return X.yrow(b, X.last(k + 1)); }, okb, vecw, part);
}

// fix-up of the group's other separators (unless FIX is false: done before, on MFMA), then
// its local backward chain xi_c = z'_c - U'_c xi_{c+1} (the group's last separator starts it)
template <typename T, int D, bool FIX>
__device__ __forceinline__ void sep_fix_bwd_local(const SolveArgs<T>& a, const Blk& B) {
    SEPK_PROLOGUE_N(FIX ? SepRB<T>::RB : SepLocalRB<T>::RB)
    const int g = B.y, c0 = X.first(g), c1 = X.last(g);
    if (FIX && g >= 1) {
        V vf[RB];
        vecs_at(X.last(g - 1), vf);
        sep_fix<T, RB>(c1 - c0, vf,
                       [&](int k) { return X.prop(c0 + k, 0); },
                       [&](int k, int b) { return X.yrow(b, c0 + k); }, okb, vecw);
    }
    V v0[RB];
    vecs_at(c1, v0);
    if constexpr (!FIX && std::is_same<T, float>::value)
        sep_chain<T, D, RB, true>(c1 - c0, true, v0, T(-1),
                                  [&](int k) { return a.Fw + ((size_t)(c1 - 1 - k) * 4 + 1) * BLK; },
                                  [&](int k, int b) { return X.yrow(b, c1 - 1 - k); }, okb, vecw, part);
    else
        sep_chain<T, D, RB>(c1 - c0, true, v0, T(-1),
                            [&](int k) { return fslot(a, X.sep(c1 - 1 - k), 2); },
                            [&](int k, int b) { return X.yrow(b, c1 - 1 - k); }, okb, vecw, part);
}

// chain over the groups' first separators: x_{first g} = xi_{first g} + Psi_{first g} x_{first g+1}
template <typename T, int D>
__device__ __forceinline__ void sep_bwd_top(const SolveArgs<T>& a, const Blk& B) {
    SEPK_PROLOGUE
    V v0[RB];
    vecs_at(X.first(a.G - 1), v0);
    if constexpr (std::is_same<T, float>::value)
        sep_chain<T, D, RB, true>(a.G - 1, true, v0, T(1),
                                  [&](int k) { return a.Fw + ((size_t)X.first(a.G - 2 - k) * 4 + 3) * BLK; },
                                  [&](int k, int b) { return X.yrow(b, X.first(a.G - 2 - k)); }, okb, vecw, part);
    else
        sep_chain<T, D, RB>(a.G - 1, true, v0, T(1),
                            [&](int k) { return X.prop(X.first(a.G - 2 - k), 1); },
                            [&](int k, int b) { return X.yrow(b, X.first(a.G - 2 - k)); }, okb, vecw, part);
}

// fix-up of the group's other separators: x_c = xi_c + Psi_c x_{first g+1}
template <typename T, int D>
__device__ __forceinline__ void sep_bwd_fix(const SolveArgs<T>& a, const Blk& B) {
    SEPK_PROLOGUE
    const int g = B.y, c0 = X.first(g), c1 = X.last(g);
    V vf[RB];
    vecs_at(X.first(g + 1), vf);
    sep_fix<T, RB>(c1 - c0, vf,
                   [&](int k) { return X.prop(c0 + 1 + k, 1); },
                   [&](int k, int b) { return X.yrow(b, c0 + 1 + k); }, okb, vecw);
}
#undef SEPK_PROLOGUE
#undef SEPK_PROLOGUE_N
// The separators' independent products for 16 right-hand sides at a time on MFMA (complex64):
//   MODE 0  a_c = G'_c r^_c for every separator c (the local forward chains' right-hand sides)
//   MODE 1  z'_c += Phi_c z'_{last g-1} for the separators of group g >= 1 but its last
//   MODE 2  x_c += Psi_c x_{first g+1} for the separators of group g < G - 1 but its first
// Grid (separators, right-hand-side groups).  Each workgroup stages its 64 x 16 operand in
// LDS and forms one (64 x 64) by (64 x 16) product in four real products (three lose
// accuracy that the iteration counts of the complex64 solves feel), so a block is read
// once per 16 right-hand sides (the per-right-hand-side workgroups of the chains read it once
// each, which makes these products bound by the CU's load bandwidth).  A workgroup writes only
// its own separator and reads only separators that no workgroup of the launch writes.
template <int MODE>
__device__ __forceinline__ void sep_par_mfma(const SolveArgs<float>& a, const Blk& B) {
    using V = float2;
    __shared__ V X[WP][17];
    const int ns = a.P - 1, c = B.x, g = c / a.q;
    const int c0 = g * a.q, c1 = min(c0 + a.q, ns) - 1;
    if (MODE == 1 && (g < 1 || c == c1)) return;
    if (MODE == 2 && (g >= a.G - 1 || c == c0)) return;
    const int sr = c * a.m + a.m - 1;                                   // the separator's row
    const int so = MODE == 1 ? (c0 - 1) * a.m + a.m - 1 : (c1 + 1) * a.m + a.m - 1;   // operand's
    const V* M = MODE == 0 ? fslot(a, sr, 0) : a.Fs + ((size_t)c * 2 + (MODE == 1 ? 0 : 1)) * BLK;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, n = lane & 15, q4 = lane >> 4;
    const int rbase = B.y * 16;
    // every load of the workgroup is issued before the first use: the A operands, then the
    // operand tile (four passes of 256 threads; branch-free, clamped addresses)
    V gA[16];
    const V* F = M + 16 * w + n;
#pragma unroll
    for (int s = 0; s < 16; ++s) gA[s] = F[(4 * s + q4) * WP];
    constexpr int NP = 16 * WP / NT;
    RawRhs raw[NP];
    V ym[NP], yp[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int idx = threadIdx.x + p * NT, q = idx >> 6, k = idx & (WP - 1), r = rbase + q;
        const V* Yr = a.Yw + (size_t)(r < a.nrhs ? r : a.nrhs - 1) * a.Ny * WP + k;
        if (MODE == 0) {
            raw[p] = load_raw(a.io, r, sr, k, a.Ny, a.nrhs, a.W);
            ym[p] = Yr[(size_t)(sr - 1) * WP];
            yp[p] = Yr[(size_t)(sr + 1) * WP];
        } else {
            ym[p] = Yr[(size_t)so * WP];
        }
    }
    // the fix-ups add to this lane's four entries of the separator
    const int rn = rbase + n;
    V* y = a.Yw + ((size_t)(rn < a.nrhs ? rn : a.nrhs - 1) * a.Ny + sr) * WP + 16 * w + 4 * q4;
    V yold[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) yold[u] = MODE == 0 ? make_float2(0.f, 0.f) : y[u];
    const double2 cys = a.cy[sr], bys = a.by[sr];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int idx = threadIdx.x + p * NT, q = idx >> 6, k = idx & (WP - 1);
        V v = make_float2(0.f, 0.f);
        if (rbase + q < a.nrhs && k < a.W) {
            if (MODE == 0) {
                v = combine<float>(a.io, raw[p]);
                v = csub(v, cmul(ccast<V>(cys), ym[p]));
                v = csub(v, cmul(ccast<V>(bys), yp[p]));
            } else {
                v = ym[p];
            }
        }
        X[k][q] = v;
    }
    __syncthreads();
    V xb[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) xb[s] = X[4 * s + q4][n];
    __builtin_amdgcn_sched_barrier(0);
    mf4 aR = {0.f, 0.f, 0.f, 0.f}, aI = aR;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const V g4 = gA[s];
        const V x = xb[s];
        aR = __builtin_amdgcn_mfma_f32_16x16x4f32(g4.x, x.x, aR, 0, 0, 0);
        aI = __builtin_amdgcn_mfma_f32_16x16x4f32(g4.x, x.y, aI, 0, 0, 0);
        aR = __builtin_amdgcn_mfma_f32_16x16x4f32(-g4.y, x.y, aR, 0, 0, 0);
        aI = __builtin_amdgcn_mfma_f32_16x16x4f32(g4.y, x.x, aI, 0, 0, 0);
    }
    if (rn >= a.nrhs) return;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const V v = make_float2(aR[u], aI[u]);
        y[u] = MODE == 0 ? v : cadd(yold[u], v);
    }
}

template <int MODE>
__global__ void __launch_bounds__(NT) k_sep_par_mfma(SolveArgs<float> a) { sep_par_mfma<MODE>(a, own_blk()); }
template <int MODE>
__global__ void __launch_bounds__(NT) k_sep_par_mfma_multi(MultiArgs<float> m) {
    int k;
    Blk b;
    if (multi_blk(m, k, b)) sep_par_mfma<MODE>(m.a[k], b);
}

template <typename T, int D, bool SETUP = true>
__global__ void __launch_bounds__(NT) k_sep_fwd_local(SolveArgs<T> a) { sep_fwd_local<T, D, SETUP>(a, own_blk()); }
template <typename T, int D, bool SETUP = true>
__global__ void __launch_bounds__(NT) k_sep_fwd_local_multi(MultiArgs<T> m) {
    int k;
    Blk b;
    if (multi_blk(m, k, b)) sep_fwd_local<T, D, SETUP>(m.a[k], b);
}
template <typename T, int D>
__global__ void __launch_bounds__(NT) k_sep_fwd_top(SolveArgs<T> a) { sep_fwd_top<T, D>(a, own_blk()); }
template <typename T, int D>
__global__ void __launch_bounds__(NT) k_sep_fwd_top_multi(MultiArgs<T> m) {
    int k;
    Blk b;
    if (multi_blk(m, k, b)) sep_fwd_top<T, D>(m.a[k], b);
}
template <typename T, int D, bool FIX = true>
__global__ void __launch_bounds__(NT) k_sep_fix_bwd_local(SolveArgs<T> a) { sep_fix_bwd_local<T, D, FIX>(a, own_blk()); }
template <typename T, int D, bool FIX = true>
__global__ void __launch_bounds__(NT) k_sep_fix_bwd_local_multi(MultiArgs<T> m) {
    int k;
    Blk b;
    if (multi_blk(m, k, b)) sep_fix_bwd_local<T, D, FIX>(m.a[k], b);
}
template <typename T, int D>
__global__ void __launch_bounds__(NT) k_sep_bwd_top(SolveArgs<T> a) { sep_bwd_top<T, D>(a, own_blk()); }
template <typename T, int D>
__global__ void __launch_bounds__(NT) k_sep_bwd_top_multi(MultiArgs<T> m) {
    int k;
    Blk b;
    if (multi_blk(m, k, b)) sep_bwd_top<T, D>(m.a[k], b);
}
template <typename T, int D>
__global__ void __launch_bounds__(NT) k_sep_bwd_fix(SolveArgs<T> a) { sep_bwd_fix<T, D>(a, own_blk()); }
template <typename T, int D>
__global__ void __launch_bounds__(NT) k_sep_bwd_fix_multi(MultiArgs<T> m) {
    int k;
    Blk b;
    if (multi_blk(m, k, b)) sep_bwd_fix<T, D>(m.a[k], b);
}

// ---------------------------------------------------------------- phase C (all columns)
template <typename T, int R>
__global__ void __launch_bounds__(NT) k_phase_c(SolveArgs<T> a) {
    using V = cplx<T>;
    constexpr int G = 4, U = R / G;
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
        const int r = rbase + g + G * u;
        // clamped load, component-wise select (a select of whole values goes through scratch)
        const bool rok = r < a.nrhs;
        const V xl = a.Yw[((size_t)(rok ? r : 0) * a.Ny + l) * WP + i];
        x[u] = cmk<V>(rok ? xl.x : T(0), rok ? xl.y : T(0));
        V xa = zero, xb = zero;
        if (r < a.nrhs) {
            if (top) xa = a.Yw[((size_t)r * a.Ny + (c * a.m - 1)) * WP + i];
            if (bot) xb = a.Yw[((size_t)r * a.Ny + (c * a.m + a.m - 1)) * WP + i];
        }
        va[i][g + G * u] = xa;
        vb[i][g + G * u] = xb;
    }
    __syncthreads();
    if (top || bot) {
        V acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = zero;
        if (top) matvec<T, R, G>(acc, fslot(a, l, 1), va, a.W, i, g);
        if (bot) matvec<T, R, G>(acc, fslot(a, l, 2), vb, a.W, i, g);
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = csub(x[u], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int r = rbase + g + G * u;
        if (r < a.nrhs && i < a.W) scatter<T>(a, r, l, i, x[u]);
    }
}

// ---------------------------------------------------------------- phase C (all columns), MFMA
// complex64: per chunk and group of 16 right-hand sides, x_l = y_l - [X~_l Y~_l] [x_a; x_b]
// for every row l of the chunk (the separator closing it is final after phase B and only
// copied), one (64 x 128) by (128 x 16) product per row on v_mfma_f32_16x16x4f32 in three
// real products.  The chunk's two separator vectors are the B operands of every row and stay
// in registers; each lane loads its A operands (A[16w + n][4s + q4] of X~_l, then of Y~_l)
// straight from global memory.  The 64 x 16 result is transposed through LDS so that the
// scatter writes whole rows of one right-hand side (consecutive x positions) instead of
// four-element pieces of sixteen right-hand sides.  Grid (chunks, right-hand-side groups,
// row groups): row group z takes the chunk's rows z, z + gridDim.z, ...
__device__ __forceinline__ void phase_c_mfma(const SolveArgs<float>& a, const Blk& B) {
    using V = float2;
    __shared__ V X[2 * WP][16];
    __shared__ V O[16][WP + 1];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, n = lane & 15, q4 = lane >> 4;
    const int c = B.x, rbase = B.y * 16;
    const int r0 = c * a.m;
    const bool has_a = c > 0, has_b = c < a.P - 1;
    const int r1 = has_b ? c * a.m + a.m - 1 : a.Ny;     // separator closing the chunk, or Ny
    const int nrow = r1 - r0 + (has_b ? 1 : 0);
    const V zero = make_float2(0.f, 0.f);
    for (int idx = t; idx < 2 * WP * 16; idx += NT) {
        const int k = idx >> 4, q = idx & 15, r = rbase + q, kk = k & (WP - 1);
        V v = zero;
        if (r < a.nrhs && kk < a.W) {
            if (k < WP) {
                if (has_a) v = a.Yw[((size_t)r * a.Ny + (r0 - 1)) * WP + kk];
            } else if (has_b) {
                v = a.Yw[((size_t)r * a.Ny + r1) * WP + kk];
            }
        }
        X[k][q] = v;
    }
    __syncthreads();
    float xr[32], xi[32], xs[32];
#pragma unroll
    for (int s = 0; s < 32; ++s) {
        const V v = X[4 * s + q4][n];
        xr[s] = v.x; xi[s] = v.y; xs[s] = v.x + v.y;
    }
    const int rn = rbase + n;
    const int qrow = 16 * w + 4 * q4;
    const size_t ybase = (size_t)(rn < a.nrhs ? rn : 0) * a.Ny * WP + qrow;
    for (int j = B.z; j < nrow; j += B.nz) {
        const int l = r0 + j;
        mf4 m1 = {0.f, 0.f, 0.f, 0.f}, m2 = m1, m3 = m1;
        if (!(has_b && l == r1)) {
            if (has_a) {
                const V* F = fslot(a, l, 1) + 16 * w + n;
#pragma unroll
                for (int s = 0; s < 16; ++s) {
                    const V g = F[(4 * s + q4) * WP];
                    m1 = __builtin_amdgcn_mfma_f32_16x16x4f32(g.x, xr[s], m1, 0, 0, 0);
                    m2 = __builtin_amdgcn_mfma_f32_16x16x4f32(g.y, xi[s], m2, 0, 0, 0);
                    m3 = __builtin_amdgcn_mfma_f32_16x16x4f32(g.x + g.y, xs[s], m3, 0, 0, 0);
                }
            }
            if (has_b) {
                const V* F = fslot(a, l, 2) + 16 * w + n;
#pragma unroll
                for (int s = 0; s < 16; ++s) {
                    const V g = F[(4 * s + q4) * WP];
                    m1 = __builtin_amdgcn_mfma_f32_16x16x4f32(g.x, xr[16 + s], m1, 0, 0, 0);
                    m2 = __builtin_amdgcn_mfma_f32_16x16x4f32(g.y, xi[16 + s], m2, 0, 0, 0);
                    m3 = __builtin_amdgcn_mfma_f32_16x16x4f32(g.x + g.y, xs[16 + s], m3, 0, 0, 0);
                }
            }
        }
        V y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) y[u] = a.Yw[ybase + (size_t)l * WP + u];
        __syncthreads();                                  // the previous row's scatter has read O
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float p1 = m1[u], p2 = m2[u], p3 = m3[u];
            O[n][qrow + u] = make_float2(y[u].x - (p1 - p2), y[u].y - (p3 - p1 - p2));
        }
        __syncthreads();
        for (int idx = t; idx < 16 * WP; idx += NT) {
            const int q = idx >> 6, i = idx & (WP - 1), r = rbase + q;
            if (r < a.nrhs && i < a.W) scatter<float>(a, r, l, i, O[q][i]);
        }
    }
}
__global__ void __launch_bounds__(NT) k_phase_c_mfma(SolveArgs<float> a) { phase_c_mfma(a, own_blk()); }
__global__ void __launch_bounds__(NT) k_phase_c_mfma_multi(MultiArgs<float> m) {
    int k;
    Blk b;
    if (multi_blk(m, k, b)) phase_c_mfma(m.a[k], b);
}

// ---------------------------------------------------------------- phase C (target columns)
// Only the 8 compact columns tcol[] of the strip; thread = (slot = t / 32, rhs = t % 32);
// ROWS consecutive rows per workgroup share the separator vectors of their chunk.
constexpr int CT_ROWS = 8;

template <typename T>
__global__ void __launch_bounds__(NT) k_phase_c_targets(SolveArgs<T> a) {
    using V = cplx<T>;
    constexpr int RC = 32;
    __shared__ V va[WP][RC];
    __shared__ V vb[WP][RC];
    __shared__ V fr[16][WP];
    const int t = threadIdx.x, rbase = blockIdx.y * RC;
    const int sl = t / RC, rr = t % RC, r = rbase + rr;
    const int q = a.tcol[sl];
    const V zero = cmk<V>(0, 0);
    const int l0 = blockIdx.x * CT_ROWS, l1 = min(a.Ny, l0 + CT_ROWS);
    int loaded = -1;
    for (int l = l0; l < l1; ++l) {
        const int c = l / a.m;
        if (c != loaded) {                       // uniform over the workgroup
            __syncthreads();
            for (int idx = t; idx < WP * RC; idx += NT) {
                const int k = idx / RC, q2 = idx % RC, r2 = rbase + q2;
                V xa = zero, xb = zero;
                if (r2 < a.nrhs && k < a.W) {
                    if (c > 0) xa = a.Yw[((size_t)r2 * a.Ny + (c * a.m - 1)) * WP + k];
                    if (c < a.P - 1) xb = a.Yw[((size_t)r2 * a.Ny + (c * a.m + a.m - 1)) * WP + k];
                }
                va[k][q2] = xa;
                vb[k][q2] = xb;
            }
            __syncthreads();
            loaded = c;
        }
        const bool is_sep = (c < a.P - 1) && (l == c * a.m + a.m - 1);
        // the 2 x 8 compact spike rows of row l (zero outside the strip width)
        const V* src = a.Fc + (size_t)l * 2 * 8 * WP;
        for (int idx = t; idx < 2 * 8 * WP; idx += NT) fr[idx / WP][idx % WP] = src[idx];
        __syncthreads();
        if (q >= 0 && r < a.nrhs) {
            V x = a.Yw[((size_t)r * a.Ny + l) * WP + q];
            if (!is_sep) {
                V acc = zero;
#pragma unroll 16
                for (int k = 0; k < WP; ++k) {
                    cfma(acc, fr[sl][k], va[k][rr]);
                    cfma(acc, fr[8 + sl][k], vb[k][rr]);
                }
                x = csub(x, acc);
            }
            scatter<T>(a, r, l, q, x);
        }
        __syncthreads();
    }
}

// complex64 target columns per chunk as one small product on v_mfma_f32_16x16x4f32:
// rows (l, t) of the chunk's interior rows l and the 8 target columns t, columns 16
// right-hand sides, k over [x_above; x_below] (128): out = Fc(l, t, :) [xa; xb], x = y - out.
// Grid (chunks, right-hand-side groups of 16, tile groups); wave w of tile group z takes row
// tiles w + 4 z, w + 4 z + 4 gridDim.z, ...  Every workgroup stages the chunk's two separator
// vectors; the separator row that closes the chunk is copied (its x is final after phase B)
// by tile group 0.
__device__ __forceinline__ void phase_c_targets_mfma(const SolveArgs<float>& a, const Blk& B) {
    using V = float2;
    __shared__ V X[2 * WP][17];
    __shared__ V XF[2][WP][17];
    __shared__ int tcs[8];                 // the target columns (the tiles' output addresses)
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, n = lane & 15, q4 = lane >> 4;
    const int c = B.x, rbase = B.y * 16;
    const int r0 = c * a.m;
    const int r1 = (c < a.P - 1) ? c * a.m + a.m - 1 : a.Ny;
    const int nr = r1 - r0;
    const bool has_a = c > 0, has_b = c < a.P - 1;
    // The two-level separator solve leaves the fix-up x_s = xi_s + Psi_s x_{first(g+1)} of the
    // separators that are not the first of their group g < G-1 to this kernel: each chunk
    // applies it to its own two separators (side 0 above, side 1 below).
    bool fix[2];
    int sfirst[2], sidx[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int cs = side ? c : c - 1;
        const int g = cs >= 0 && a.q > 0 ? cs / a.q : 0;
        sidx[side] = cs;
        fix[side] = a.io.targets_only && a.G >= 2 && a.Fs && a.P > 2 && (side ? has_b : has_a) &&
                    g < a.G - 1 && cs != g * a.q;
        sfirst[side] = (g + 1) * a.q;
    }
    // branch-free staging: every lane loads (a clamped address) and keeps or drops the value
    {
        V xv[8], fv[8];
        bool keepv[8], keepf[8];
        // element e: right-hand side j = e / 128, k = e % 128 (consecutive lanes read
        // consecutive columns of one right-hand side's row)
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = t + NT * u;
            const int k = e & (2 * WP - 1), j = e >> 7, r = rbase + j, kk = k & (WP - 1);
            const bool above = k < WP;
            keepv[u] = r < a.nrhs && kk < a.W && (above ? has_a : has_b);
            const int row = above ? (has_a ? r0 - 1 : r0) : (has_b ? r1 : r0);
            const size_t rr = (size_t)(r < a.nrhs ? r : 0) * a.Ny;
            xv[u] = a.Yw[(rr + row) * WP + kk];
            const int side = above ? 0 : 1;
            keepf[u] = keepv[u] && fix[side];
            // a dropped value reads row 0: an address the compiler cannot equate with xv's,
            // which would make it reuse xv behind a wait for every element
            const int frow = fix[side] ? sfirst[side] * a.m + a.m - 1 : 0;
            fv[u] = a.Yw[(rr + frow) * WP + kk];
        }
        const int tc = a.tcol[t & 7];          // waited for with the loads above
        if (t < 8) tcs[t] = tc;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = t + NT * u;
            const int k = e & (2 * WP - 1), j = e >> 7;
            X[k][j] = make_float2(keepv[u] ? xv[u].x : 0.f, keepv[u] ? xv[u].y : 0.f);
            XF[k >> 6][k & (WP - 1)][j] = make_float2(keepf[u] ? fv[u].x : 0.f, keepf[u] ? fv[u].y : 0.f);
        }
    }
    __syncthreads();
    if (fix[0] || fix[1]) {
        // X[side] += Psi_s XF[side] (64 x 64 by 64 x 16 on MFMA in four real products;
        // wave w: rows 16 w ..); both sides' blocks are loaded before either product
        V g[2][16];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const V* Ps = a.Fs + ((size_t)(fix[side] ? sidx[side] : 0) * 2 + 1) * BLK + 16 * w + n;
#pragma unroll
            for (int s4 = 0; s4 < 16; ++s4) g[side][s4] = Ps[(size_t)(4 * s4 + q4) * WP];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            if (!fix[side]) continue;
            mf4 aR = {0.f, 0.f, 0.f, 0.f}, aI = aR;
#pragma unroll
            for (int s4 = 0; s4 < 16; ++s4) {
                const V g0 = g[side][s4];
                const V v0 = XF[side][4 * s4 + q4][n];
                aR = __builtin_amdgcn_mfma_f32_16x16x4f32(g0.x, v0.x, aR, 0, 0, 0);
                aI = __builtin_amdgcn_mfma_f32_16x16x4f32(g0.x, v0.y, aI, 0, 0, 0);
                aR = __builtin_amdgcn_mfma_f32_16x16x4f32(-g0.y, v0.y, aR, 0, 0, 0);
                aI = __builtin_amdgcn_mfma_f32_16x16x4f32(g0.y, v0.x, aI, 0, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                V& xr = X[WP * side + 16 * w + 4 * q4 + j][n];
                xr = make_float2(xr.x + aR[j], xr.y + aI[j]);
            }
        }
        __syncthreads();
    }
    const int rn = rbase + n;
    const int nrows = nr * 8, ntile = (nrows + 15) / 16;
    // k-step s of a side takes the column kc(s) = 8 (s / 2) + 2 q4 + s % 2 in this lane, so
    // that the lane's two columns of k-steps 2i, 2i + 1 are adjacent and come in one 16-byte
    // load (each load instruction reads 64 contiguous bytes of 16 compact rows).  The B panel
    // of every tile, [x_above; x_below], in the same order:
    V vb[32];
#pragma unroll
    for (int s4 = 0; s4 < 32; ++s4) vb[s4] = X[WP * (s4 >> 4) + 8 * ((s4 & 15) >> 1) + 2 * q4 + (s4 & 1)][n];
    for (int tile = w + 4 * B.z; tile < ntile; tile += 4 * B.nz) {
        // A operands: row rho = 16 tile + n (clamped), columns kc(s) of both sides
        const int rho = min(16 * tile + n, nrows - 1);
        const int l = r0 + (rho >> 3), tt = rho & 7;
        const float4* fa = reinterpret_cast<const float4*>(a.Fc + ((size_t)(l * 2 + 0) * 8 + tt) * WP) + q4;
        const float4* fb = reinterpret_cast<const float4*>(a.Fc + ((size_t)(l * 2 + 1) * 8 + tt) * WP) + q4;
        V g[32];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float4 va = fa[4 * i], vb4 = fb[4 * i];
            g[2 * i] = make_float2(va.x, va.y);
            g[2 * i + 1] = make_float2(va.z, va.w);
            g[16 + 2 * i] = make_float2(vb4.x, vb4.y);
            g[16 + 2 * i + 1] = make_float2(vb4.z, vb4.w);
        }
        // the y values of this lane's four outputs, loaded before the products (the
        // stores of the outputs below could alias them, so they cannot move up by themselves)
        V y[4];
        int qo[4], lo4[4];
        bool ok[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int ro = 16 * tile + 4 * q4 + j;
            const int roc = ro < nrows ? ro : nrows - 1;
            lo4[j] = r0 + (roc >> 3);
            qo[j] = tcs[roc & 7];
            ok[j] = ro < nrows && qo[j] >= 0 && rn < a.nrhs;
            const size_t yi = ((size_t)(rn < a.nrhs ? rn : 0) * a.Ny + lo4[j]) * WP + (qo[j] >= 0 ? qo[j] : 0);
            y[j] = a.Yw[yi];
        }
        __builtin_amdgcn_sched_barrier(0);       // every operand of the tile in flight first
        // four real products per complex one (the three-product form costs accuracy here)
        mf4 aR0 = {0.f, 0.f, 0.f, 0.f}, aI0 = aR0, aR1 = aR0, aI1 = aR0;
#pragma unroll
        for (int s4 = 0; s4 < 32; s4 += 2) {
            const V g0 = g[s4], g1 = g[s4 + 1];
            const V v0 = vb[s4], v1 = vb[s4 + 1];
            aR0 = __builtin_amdgcn_mfma_f32_16x16x4f32(g0.x, v0.x, aR0, 0, 0, 0);
            aI0 = __builtin_amdgcn_mfma_f32_16x16x4f32(g0.x, v0.y, aI0, 0, 0, 0);
            aR1 = __builtin_amdgcn_mfma_f32_16x16x4f32(g1.x, v1.x, aR1, 0, 0, 0);
            aI1 = __builtin_amdgcn_mfma_f32_16x16x4f32(g1.x, v1.y, aI1, 0, 0, 0);
            aR0 = __builtin_amdgcn_mfma_f32_16x16x4f32(-g0.y, v0.y, aR0, 0, 0, 0);
            aI0 = __builtin_amdgcn_mfma_f32_16x16x4f32(g0.y, v0.x, aI0, 0, 0, 0);
            aR1 = __builtin_amdgcn_mfma_f32_16x16x4f32(-g1.y, v1.y, aR1, 0, 0, 0);
            aI1 = __builtin_amdgcn_mfma_f32_16x16x4f32(g1.y, v1.x, aI1, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (ok[j]) {
                const V x = make_float2(y[j].x - (aR0[j] + aR1[j]), y[j].y - (aI0[j] + aI1[j]));
                scatter<float>(a, rn, lo4[j], qo[j], x);
            }
        }
    }
    // the separator row closing this chunk (its x, fixed up above if needed, is in X)
    if (has_b && B.z == 0 && t < 8 * 16) {
        const int tt = t >> 4, r = rbase + (t & 15), q = tcs[tt];
        if (q >= 0 && r < a.nrhs) scatter<float>(a, r, r1, q, X[WP + q][t & 15]);
    }
}
__global__ void __launch_bounds__(NT) k_phase_c_targets_mfma(SolveArgs<float> a) {
    phase_c_targets_mfma(a, own_blk());
}
__global__ void __launch_bounds__(NT) k_phase_c_targets_mfma_multi(MultiArgs<float> m) {
    int k;
    Blk b;
    if (multi_blk(m, k, b)) phase_c_targets_mfma(m.a[k], b);
}

template <typename T> struct Depth { static constexpr int D = 2; };
template <> struct Depth<float> { static constexpr int D = 4; };

template <typename T, int R>
void launch_phase_a(const SolveArgs<T>& a, int RG, hipStream_t st) {
    hipLaunchKernelGGL((k_phase_a<T, R>), dim3(a.P, RG), dim3(NT), 0, st, a);
}
template <>
void launch_phase_a<float, 16>(const SolveArgs<float>& a, int RG, hipStream_t st) {
    hipLaunchKernelGGL(k_phase_a_mfma<2>, dim3(a.P, RG), dim3(NT), 0, st, a);
}

template <typename T, int R>
hipError_t run(const SolveArgs<T>& a, bool targets, hipStream_t st, KTimer* kt) {
    const int RG = (a.nrhs + R - 1) / R;
    if (kt) kt->begin(K_PHASE_A, st);
    launch_phase_a<T, R>(a, RG, st);
    if (kt) kt->end(K_PHASE_A, st);
    if (a.P > 1) {
        if (kt) kt->begin(K_PHASE_B, st);
        if (a.P > 2 && a.G >= 2 && a.Fs) {
            constexpr int DS = Depth<T>::D;
            const unsigned nr = (unsigned)((a.nrhs + SepRB<T>::RB - 1) / SepRB<T>::RB);
            if constexpr (std::is_same<T, float>::value) {
                // the independent products on MFMA, the chains one right-hand side per
                // workgroup; targets-only solves fix the separators up inside phase C
                const dim3 gp(a.P - 1, (a.nrhs + 15) / 16);
                const unsigned nl = (unsigned)((a.nrhs + SepLocalRB<T>::RB - 1) / SepLocalRB<T>::RB);
                hipLaunchKernelGGL(k_sep_par_mfma<0>, gp, dim3(NT), 0, st, a);
                hipLaunchKernelGGL((k_sep_fwd_local<T, DS, false>), dim3(nl, a.G), dim3(NT), 0, st, a);
                hipLaunchKernelGGL((k_sep_fwd_top<T, DS>), dim3(nr), dim3(NT), 0, st, a);
                hipLaunchKernelGGL(k_sep_par_mfma<1>, gp, dim3(NT), 0, st, a);
                hipLaunchKernelGGL((k_sep_fix_bwd_local<T, DS, false>), dim3(nl, a.G), dim3(NT), 0, st, a);
                hipLaunchKernelGGL((k_sep_bwd_top<T, DS>), dim3(nr), dim3(NT), 0, st, a);
                if (!targets) hipLaunchKernelGGL(k_sep_par_mfma<2>, gp, dim3(NT), 0, st, a);
            } else {
                // the local forward chains form their own right-hand sides a_c
                hipLaunchKernelGGL((k_sep_fwd_local<T, DS>), dim3(nr, a.G), dim3(NT), 0, st, a);
                hipLaunchKernelGGL((k_sep_fwd_top<T, DS>), dim3(nr), dim3(NT), 0, st, a);
                hipLaunchKernelGGL((k_sep_fix_bwd_local<T, DS>), dim3(nr, a.G), dim3(NT), 0, st, a);
                hipLaunchKernelGGL((k_sep_bwd_top<T, DS>), dim3(nr), dim3(NT), 0, st, a);
                hipLaunchKernelGGL((k_sep_bwd_fix<T, DS>), dim3(nr, a.G - 1), dim3(NT), 0, st, a);
            }
        } else {
            hipLaunchKernelGGL((k_phase_b0<T, R>), dim3(a.P - 1, RG), dim3(NT), 0, st, a);
        }
        if (a.P > 2 && !(a.G >= 2 && a.Fs)) {
            if (a.P - 1 <= ZMAX)
                hipLaunchKernelGGL((k_phase_b<T, Depth<T>::D, true>), dim3(a.nrhs), dim3(NT), 0, st, a);
            else
                hipLaunchKernelGGL((k_phase_b<T, Depth<T>::D, false>), dim3(a.nrhs), dim3(NT), 0, st, a);
        }
        if (kt) kt->end(K_PHASE_B, st);
    }
    if (kt) kt->begin(K_PHASE_C, st);
    if (targets) {
        if constexpr (std::is_same<T, float>::value) {
            // the 16-row tiles of a chunk are spread over TS workgroups (two tiles per wave
            // at m = 32: measured faster than one or four)
            const int tiles = ((a.m - 1) * 8 + 15) / 16;
            const int TS = std::min(8, std::max(1, (tiles + 7) / 8));      // targets_groups
            hipLaunchKernelGGL(k_phase_c_targets_mfma, dim3(a.P, (a.nrhs + 15) / 16, TS), dim3(NT), 0, st, a);
        }
        else
            hipLaunchKernelGGL((k_phase_c_targets<T>), dim3((a.Ny + CT_ROWS - 1) / CT_ROWS, (a.nrhs + 31) / 32),
                               dim3(NT), 0, st, a);
    }
    else if constexpr (std::is_same<T, float>::value) {
        // about four workgroups per CU: row groups split each chunk's rows (phase_c_groups)
        const int per = a.P * ((a.nrhs + 15) / 16);
        const int TS = std::max(1, std::min(std::min(8, a.m), (1024 + per - 1) / per));
        hipLaunchKernelGGL(k_phase_c_mfma, dim3(a.P, (a.nrhs + 15) / 16, TS), dim3(NT), 0, st, a);
    } else
        hipLaunchKernelGGL((k_phase_c<T, R>), dim3(a.Ny, RG), dim3(NT), 0, st, a);
    if (kt) kt->end(K_PHASE_C, st);
    return hipGetLastError();
}

template <typename T>
SolveArgs<T> solve_args(const DevTables& t, const Geom& g, const Chunks& ch, int s, int fs,
                        const cplx<T>* F, const cplx<T>* Fc, const cplx<T>* Fs, const cplx<T>* Fa,
                        const cplx<T>* Fw, cplx<T>* Yw, int nrhs, const IOSpec& io) {
    SolveArgs<T> a;
    a.F = F + (size_t)fs * g.Ny * NSLOT * BLK;
    a.Fs = Fs ? Fs + (size_t)fs * (ch.P - 1) * 2 * BLK : nullptr;
    a.Fa = Fa ? Fa + (size_t)fs * g.Ny * BLK : nullptr;
    a.Fw = Fw ? Fw + (size_t)fs * (ch.P - 1) * 4 * BLK : nullptr;
    a.q = ch.q;
    a.G = ch.G;
    a.Fc = Fc ? Fc + (size_t)fs * g.Ny * 2 * 8 * WP : nullptr;
    a.tcol = t.tcol + s * 8;
    a.Yw = Yw;
    a.cy = t.cy;
    a.by = t.by;
    a.io = io;
    if (!Fc) a.io.targets_only = 0;     // without compact rows phase C reads every column
    if (!a.io.trA || !a.io.trB || a.io.q_t < 0) {   // the gather always dereferences them
        a.io.trA = a.io.trB = a.io.src;
        a.io.q_t = -1;
        a.io.coef = 0.0;
    }
    a.Ny = g.Ny;
    a.W = g.strips[s].W;
    a.m = ch.m;
    a.P = ch.P;
    a.nrhs = nrhs;
    return a;
}

}  // namespace

template <typename T>
hipError_t launch_strip_solve(const DevTables& t, const Geom& g, const Chunks& ch, int s, int fs,
                              const cplx<T>* F, const cplx<T>* Fc, const cplx<T>* Fs, const cplx<T>* Fa,
                              const cplx<T>* Fw, cplx<T>* Yw, int nrhs, const IOSpec& io, hipStream_t st,
                              KTimer* kt) {
    const SolveArgs<T> a = solve_args<T>(t, g, ch, s, fs, F, Fc, Fs, Fa, Fw, Yw, nrhs, io);
    // complex64 reads the operand-order copies: phase A on MFMA (more than 4 right-hand
    // sides) and the separator chains of the two-level solve
    if (std::is_same<T, float>::value &&
        ((nrhs > 4 && !Fa) || (ch.P > 2 && ch.G >= 2 && Fs && !Fw)))
        return hipErrorInvalidValue;
    const bool targets = a.io.targets_only != 0;
    if (nrhs <= 4) return run<T, 4>(a, targets, st, kt);
    return run<T, 16>(a, targets, st, kt);
}

namespace {
SolveArgs<float> job_args(const StripJob& j) {
    return solve_args<float>(*j.t, *j.g, *j.ch, j.s, j.fs, static_cast<const float2*>(j.F),
                             static_cast<const float2*>(j.Fc), static_cast<const float2*>(j.Fs),
                             static_cast<const float2*>(j.Fa), static_cast<const float2*>(j.Fw),
                             static_cast<float2*>(j.Yw), j.nrhs, j.io);
}
// rows of the full-column phase C per workgroup: about four workgroups per CU
int phase_c_groups(const SolveArgs<float>& a) {
    const int per = a.P * ((a.nrhs + 15) / 16);
    return std::max(1, std::min(std::min(8, a.m), (1024 + per - 1) / per));
}
int targets_groups(const SolveArgs<float>& a) {
    const int tiles = ((a.m - 1) * 8 + 15) / 16;
    return std::min(8, std::max(1, (tiles + 7) / 8));
}
}  // namespace

bool strip_jobs_fusable(const StripJob* jobs, int n) {
    if (n < 2 || n > MULTI_MAX) return false;
    int targets = -1;
    for (int k = 0; k < n; ++k) {
        const StripJob& j = jobs[k];
        if (!j.f32 || j.g->dim != 2 || j.nrhs <= 4) return false;
        if (!(j.ch->P > 2 && j.ch->G >= 2 && j.Fs)) return false;        // two-level separators
        if (!j.Fa || !j.Fw) return false;                                // operand-order copies
        const int tk = (j.io.targets_only && j.Fc) ? 1 : 0;
        if (targets >= 0 && tk != targets) return false;
        targets = tk;
    }
    return true;
}

hipError_t launch_strip_solve_multi(const StripJob* jobs, int n, hipStream_t st, KTimer* kt) {
    if (!strip_jobs_fusable(jobs, n)) return hipErrorInvalidValue;
    MultiArgs<float> m{};
    m.n = n;
    for (int k = 0; k < n; ++k) m.a[k] = job_args(jobs[k]);
    const bool targets = m.a[0].io.targets_only != 0;
    // x blocks per problem, and per-problem y / z extents (the launch takes the largest)
    auto shape = [&](auto xper, auto yper, auto zper, dim3& grid) {
        m.xs[0] = 0;
        int my = 1, mz = 1;
        for (int k = 0; k < n; ++k) {
            m.xs[k + 1] = m.xs[k] + xper(m.a[k]);
            m.ny[k] = yper(m.a[k]);
            m.nz[k] = zper(m.a[k]);
            my = std::max(my, m.ny[k]);
            mz = std::max(mz, m.nz[k]);
        }
        grid = dim3(m.xs[n], my, mz);
    };
    auto P = [](const SolveArgs<float>& a) { return a.P; };
    auto RG = [](const SolveArgs<float>& a) { return (a.nrhs + 15) / 16; };
    auto NR = [](const SolveArgs<float>& a) { return a.nrhs; };     // one right-hand side per block
    auto NL = [](const SolveArgs<float>& a) {                       // the local chains' blocks
        return (a.nrhs + SepLocalRB<float>::RB - 1) / SepLocalRB<float>::RB;
    };
    auto G = [](const SolveArgs<float>& a) { return a.G; };
    auto NS = [](const SolveArgs<float>& a) { return a.P - 1; };      // separators
    auto one = [](const SolveArgs<float>&) { return 1; };
    constexpr int DS = Depth<float>::D;
    dim3 grid;
    if (kt) kt->begin(K_PHASE_A, st);
    shape(P, RG, one, grid);
    hipLaunchKernelGGL(k_phase_a_mfma_multi<2>, grid, dim3(NT), 0, st, m);
    if (kt) kt->end(K_PHASE_A, st);
    if (kt) kt->begin(K_PHASE_B, st);
    shape(NS, RG, one, grid);
    hipLaunchKernelGGL(k_sep_par_mfma_multi<0>, grid, dim3(NT), 0, st, m);
    shape(NL, G, one, grid);
    hipLaunchKernelGGL((k_sep_fwd_local_multi<float, DS, false>), grid, dim3(NT), 0, st, m);
    shape(NR, one, one, grid);
    hipLaunchKernelGGL((k_sep_fwd_top_multi<float, DS>), grid, dim3(NT), 0, st, m);
    shape(NS, RG, one, grid);
    hipLaunchKernelGGL(k_sep_par_mfma_multi<1>, grid, dim3(NT), 0, st, m);
    shape(NL, G, one, grid);
    hipLaunchKernelGGL((k_sep_fix_bwd_local_multi<float, DS, false>), grid, dim3(NT), 0, st, m);
    shape(NR, one, one, grid);
    hipLaunchKernelGGL((k_sep_bwd_top_multi<float, DS>), grid, dim3(NT), 0, st, m);
    if (!targets) {
        shape(NS, RG, one, grid);
        hipLaunchKernelGGL(k_sep_par_mfma_multi<2>, grid, dim3(NT), 0, st, m);
    }
    if (kt) kt->end(K_PHASE_B, st);
    if (kt) kt->begin(K_PHASE_C, st);
    if (targets) {
        shape(P, RG, targets_groups, grid);
        hipLaunchKernelGGL(k_phase_c_targets_mfma_multi, grid, dim3(NT), 0, st, m);
    } else {
        shape(P, RG, phase_c_groups, grid);
        hipLaunchKernelGGL(k_phase_c_mfma_multi, grid, dim3(NT), 0, st, m);
    }
    if (kt) kt->end(K_PHASE_C, st);
    return hipGetLastError();
}

template hipError_t launch_strip_solve<float>(const DevTables&, const Geom&, const Chunks&, int, int,
                                              const float2*, const float2*, const float2*, const float2*,
                                              const float2*, float2*, int, const IOSpec&, hipStream_t, KTimer*);
template hipError_t launch_strip_solve<double>(const DevTables&, const Geom&, const Chunks&, int, int,
                                               const double2*, const double2*, const double2*,
                                               const double2*, const double2*, double2*, int, const IOSpec&,
                                               hipStream_t, KTimer*);

namespace {
// Fa[slot][row]: out[((w * 8 + i) * 64 + 16 q4 + n) * 2 + h] = G[16 w + n][8 i + 4 h + q4] of
// F[slot][row][0] (column-major: element (r, c) at c * WP + r)
__global__ void __launch_bounds__(NT) k_swizzle_a(const float2* __restrict__ F, float2* __restrict__ Fa) {
    const size_t blk = blockIdx.x;                       // slot * Ny + row
    const float2* src = F + blk * NSLOT * BLK;
    float2* dst = Fa + blk * BLK;
    for (int o = threadIdx.x; o < BLK; o += NT) {
        const int h = o & 1, lane = (o >> 1) & 63, i = (o >> 7) & 7, w = o >> 10;
        const int q4 = lane >> 4, n = lane & 15;
        dst[o] = src[(8 * i + 4 * h + q4) * WP + 16 * w + n];
    }
}
// Fw[slot][c][kind]: out[((w * 8 + j) * 64 + i) * 2 + h] = M[i][16 w + 2 j + h] for M = the
// slot-1 / slot-2 block at separator row c m + m - 1 (kind 0 / 1) or the propagator Fs[c][0 / 1]
// (kind 2 / 3)
__global__ void __launch_bounds__(NT) k_swizzle_w(const float2* __restrict__ F, const float2* __restrict__ Fs,
                                                  float2* __restrict__ Fw, int Ny, int m, int ns) {
    const int kind = blockIdx.x & 3, c = (blockIdx.x >> 2) % ns, slot = (blockIdx.x >> 2) / ns;
    const int row = c * m + m - 1;
    const float2* src = kind < 2 ? F + (((size_t)slot * Ny + row) * NSLOT + 1 + kind) * BLK
                                 : Fs + (((size_t)slot * ns + c) * 2 + (kind - 2)) * BLK;
    float2* dst = Fw + (size_t)blockIdx.x * BLK;
    for (int o = threadIdx.x; o < BLK; o += NT) {
        const int h = o & 1, i = (o >> 1) & 63, j = (o >> 7) & 7, w = o >> 10;
        dst[o] = src[(16 * w + 2 * j + h) * WP + i];
    }
}
}  // namespace

hipError_t launch_swizzle_factors(const float2* F, const float2* Fs, float2* Fa, float2* Fw,
                                  const Geom& g, const Chunks& ch, int nfac, hipStream_t st) {
    if (nfac <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_swizzle_a, dim3((unsigned)(nfac * g.Ny)), dim3(NT), 0, st, F, Fa);
    const int ns = ch.P - 1;
    if (Fw && Fs && ns > 0)
        hipLaunchKernelGGL(k_swizzle_w, dim3((unsigned)(nfac * ns * 4)), dim3(NT), 0, st, F, Fs, Fw, g.Ny,
                           ch.m, ns);
    return hipGetLastError();
}

}  // namespace helm

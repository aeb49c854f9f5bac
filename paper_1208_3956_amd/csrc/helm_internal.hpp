// Internal declarations shared by the host core and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "helm.h"

namespace helm {

// Every padded strip is at most WP columns wide; its dense y-blocks are stored as
// WP x WP column-major matrices (element (i,k) at k*WP + i), zero outside the leading
// W x W corner.
constexpr int WP = 64;
constexpr int BLK = WP * WP;
constexpr int NSLOT = 3;   // per row: G (or G'), top spike X~ (or L), bottom spike Y~ (or U')

// ---------------------------------------------------------------- complex helpers
template <typename T> struct cvec;
template <> struct cvec<float> { using type = float2; };
template <> struct cvec<double> { using type = double2; };
template <typename T> using cplx = typename cvec<T>::type;

template <typename V> __host__ __device__ inline V cmk(decltype(V{}.x) re, decltype(V{}.x) im) {
    V r; r.x = re; r.y = im; return r;
}
template <typename V> __host__ __device__ inline V cadd(V a, V b) { return cmk<V>(a.x + b.x, a.y + b.y); }
template <typename V> __host__ __device__ inline V csub(V a, V b) { return cmk<V>(a.x - b.x, a.y - b.y); }
template <typename V> __host__ __device__ inline V cmul(V a, V b) {
    return cmk<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename V> __host__ __device__ inline V cconjmul(V a, V b) {  // conj(a) * b
    return cmk<V>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// acc += a * b
template <typename V> __device__ inline void cfma(V& acc, V a, V b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}
template <typename To, typename Ti> __host__ __device__ inline To ccast(Ti a) {
    To r; r.x = a.x; r.y = a.y; return r;
}

// ---------------------------------------------------------------- geometry (host)
struct Strip {
    int a, W;              // first global column and width of the padded strip
    int core_lo, core_hi;  // D^(j)
    int dom_lo, dom_hi;    // non-pad columns (core + the extra column on the right)
    int kdn_lo, kdn_hi;    // D~^(j), kept by the downward sweep
    bool lpad, rpad;
};

struct Geom {
    int nx = 0, ny = 0, Nx = 0, Ny = 0, wout = 0, w = 0, J = 0;
    int dim = 2, nz = 0, Nz = 1;  // 3-D: nz interior points along z, Nz = nz + 2 wout
    int Bp = 0;                   // 3-D: slab block size W * Nz padded to a multiple of 64
    // rows of a field: fields are [rhs][row][x] with row = z * Ny + y
    long Nrow() const { return (long)Nz * Ny; }
    double h = 0, omega = 0, power = 2, s0 = 10, cref = 0;
    double s0i = 0;              // strength of the interface pads (strip operators only)
    std::vector<int> beta;       // J+1 entries
    std::vector<Strip> strips;
};

// y-partition of every strip into chunks of m rows whose last row is a separator
struct Chunks {
    int m = 0, P = 0;            // rows per chunk, number of chunks
    // the P-1 separators form groups of q consecutive ones (G groups, the last ragged) for
    // the two-level separator solve; G < 2 means one chain
    int q = 0, G = 0;
    int gfirst(int g) const { return g * q; }
    int glast(int g) const { return (g * q + q < P - 1 ? g * q + q : P - 1) - 1; }
    int first(int c) const { return c * m; }
    int end(int c, int Ny) const { return c < P - 1 ? c * m + m - 1 : Ny; }   // interior end
    int sep(int c) const { return c * m + m - 1; }                              // c < P-1
};

// Input gather / output scatter of one strip solve.  Strip-local column q of row l and
// right-hand side r maps to element r*rs + l*ls + (q + off) of the buffer.
struct IOSpec {
    const double2* src = nullptr;  long src_rs = 0; int src_ls = 0; int src_off = 0;
    int src_lo = 0, src_hi = 0;    // strip-local columns taken from src
    // transmission source coef * (trB - trA) added at columns q_t and q_t + 1
    const double2* trA = nullptr; const double2* trB = nullptr; int q_t = -1; double coef = 0;
    // outputs: up to two strip-local column ranges written (or accumulated) into dst; column
    // q of range k goes to dst[r * dst_rs + row * dst_ls + q + dst_off[k]]
    double2* dst = nullptr;  long dst_rs = 0; int dst_ls = 0; int dst_off[2] = {0, 0};
    int o_lo[2] = {0, 0}, o_hi[2] = {0, 0};
    int accumulate = 0;
    // outgoing traces: x[qo[0]] -> tro[0][r*Ny + l], x[qo[1]] -> tro[1][r*Ny + l]
    double2* tro0 = nullptr; double2* tro1 = nullptr; int qo0 = -1, qo1 = -1;
    // every requested column is one of the strip's 8 compact target columns: phase C may
    // compute only those (reduced form)
    int targets_only = 0;
    // columns receiving the transmission source: 2 (q_t and q_t + 1, the PML transmission)
    // or 1 (q_t only, a Robin side)
    int t_cols = 2;
};

// One strip solve of a multi-problem launch (one strip of each of several problems).
constexpr int MULTI_MAX = 8;
struct DevTables;
struct KTimer;
struct StripJob {
    const DevTables* t = nullptr;
    const Geom* g = nullptr;
    const Chunks* ch = nullptr;
    int s = 0, fs = 0;                   // strip and its factor slot
    bool f32 = false;                    // complex64 factors and workspace
    const void* F = nullptr;
    const void* Fc = nullptr;
    const void* Fs = nullptr;
    const void* Fa = nullptr;            // operand-order copies (launch_swizzle_factors)
    const void* Fw = nullptr;
    void* Yw = nullptr;
    int nrhs = 0;
    IOSpec io;
};
// The jobs run as one launch per phase: 2 to MULTI_MAX of them, all complex64 2-D strips
// with more than 4 right-hand sides on the two-level separator solve, and the same phase-C
// form (target columns or all).
bool strip_jobs_fusable(const StripJob* jobs, int n);
hipError_t launch_strip_solve_multi(const StripJob* jobs, int n, hipStream_t st, KTimer* kt);

// Strip-local column q receives the transmission source of io.
__host__ __device__ inline bool tr_col(const IOSpec& io, int q) {
    return io.q_t >= 0 && (q == io.q_t || (io.t_cols == 2 && q == io.q_t + 1));
}

// Device tables of one problem.
struct DevTables {
    double* k2 = nullptr;       // Ny*Nx
    double2* ax = nullptr;      // Nx
    double2* axh = nullptr;     // Nx+1
    double2* ay = nullptr;      // Ny
    double2* ayh = nullptr;     // Ny+1
    double2* cy = nullptr;      // Ny: coupling of row l to row l-1 (same for every column)
    double2* by = nullptr;      // Ny: coupling of row l to row l+1
    double2* sax = nullptr;     // J*WP     strip alpha_x at points
    double2* saxh = nullptr;    // J*(WP+1) strip alpha_x at half-points
    int* scol = nullptr;        // J*WP     column whose medium each strip column uses
    int* sW = nullptr;          // J        strip widths
    int* rcols = nullptr;       // 2(J-1)   residual columns beta_j - 1, beta_j
    int* redcols = nullptr;     // 2(J-1)   reduced columns beta_j, beta_j + 1
    int* tcol = nullptr;        // J*8      strip-local columns whose spike rows are kept compact
    int* bw = nullptr;          // J-1      first column beta_j - 2 of each interface window
    double* k2w = nullptr;      // Nrow*(J-1)*IWIN  k^2 on the interface windows
    double2* az = nullptr;      // Nz       (3-D) alpha_z at points
    double2* azh = nullptr;     // Nz+1     (3-D) alpha_z at half-points
    // Robin subdomains (2-D comparison method): diagonal terms of the first / last column,
    // [strip][row][2]; rho = (1 + i k h/2)/(1 - i k h/2) of every interface, [J-1][row]
    double2* srob = nullptr;
    double2* rho = nullptr;
};

// Interface windows: the reduced form only ever touches the columns beta_j - 2 .. beta_j + 2
// around each interface j = 1..J-1.  Window fields hold just those, [nrhs][Nrow][J-1][IWIN]
// (the IWIN columns of consecutive interfaces side by side in a row).
constexpr int IWIN = 5;

// ---- 3-D slabs (kernels_3d.hip)
constexpr int BP3_MAX = 8192;   // largest padded slab block

struct Fac3Args {
    int J, Ny, Nz, Nx, Bp;
    const int* sW;
    const double2* sax; const double2* saxh; const int* scol;
    const double2* ay; const double2* ayh; const double2* az; const double2* azh;
    const double2* cy; const double2* by;
    const double* k2;
    double ih2;
};

template <typename T>
struct Solve3Args {
    const cplx<T>* F;     // factors of the slab: [Ny][Bp*Bp], column-major inverses G_l
    cplx<T>* Yw;          // workspace [Ny][Bp][RP]
    cplx<T>* Tw;          // workspace 2 x [Bp][RP]: right-hand sides of the forward planes
    const double2* cy;
    const double2* by;
    IOSpec io;            // rows of src / dst are z * Ny + y; traces are [rhs][Nrow]
    int Ny, Nz, W, B, Bp, nrhs, RP;
    long Nrow;
};

// Optional per-launch event timing: launchers call begin/end around each kernel.
struct KTimer {
    virtual void begin(int cls, hipStream_t st) = 0;
    virtual void end(int cls, hipStream_t st) = 0;
    virtual ~KTimer() = default;
};
enum KClass { K_PHASE_A = 0, K_PHASE_B, K_PHASE_C, K_FACTOR_CHUNKS, K_FACTOR_SEPS, K_STENCIL,
              K_GMRES, K_OTHER, K_NCLASS };

// ---------------------------------------------------------------- kernels (launchers)
// F32 (complex64 path) receives every stored block rounded to complex64, null otherwise
hipError_t launch_factor_chunks(const DevTables& t, const Geom& g, const Chunks& ch,
                                double2* F64, float2* F32, int* err, hipStream_t st);
hipError_t launch_factor_separators(const DevTables& t, const Geom& g, const Chunks& ch,
                                    double2* F64, float2* F32, int* err, hipStream_t st);
// propagators of the two-level separator solve, Fs[s][c][2][BLK] (FP64, and rounded into
// Fs32 when it is not null): forward Phi_c = -K_c Phi_{c-1} from the first separator of each
// group on (groups 1..G-1), backward Psi_c = -U'_c Psi_{c+1} from the last one down
// (groups 0..G-2)
hipError_t launch_factor_propagators(const DevTables& t, const Geom& g, const Chunks& ch,
                                     const double2* F64, double2* Fs, float2* Fs32, hipStream_t st);
// copies of the spike rows at the 8 target columns tcol[s*8 + t] (-1 = unused) of each strip
template <typename V>
hipError_t launch_extract_targets(const V* F, V* Fc, const int* tcol, const Geom& g,
                                  const Chunks& ch, hipStream_t st);

// Operand-order copies of complex64 factor blocks, for 16-byte loads of two adjacent values
// per lane (a CU issues loads per instruction, so half the instructions move the same bytes
// in about half the time).  Fa[slot][row][BLK]: block G_l (slot 0) of every row, laid out as
// [wave w][pair i][lane][2] holding G_l[16 w + n][8 i + 4 h + q4] (lane = 16 q4 + n, h the
// half), the A operands of the phase-A products in their k-step order.  Fw[slot][c][4][BLK]:
// for separator c, the chain blocks (slot 1 and slot 2 at its row) and the propagators (Fs
// forward, backward), laid out as [wave w][pair j][row i][2] holding M[i][16 w + 2 j + h].
// Fw is written only when the factor has propagators (two-level separator solve).
hipError_t launch_swizzle_factors(const float2* F, const float2* Fs, float2* Fa, float2* Fw,
                                  const Geom& g, const Chunks& ch, int nfac, hipStream_t st);

template <typename T>
// strip s with its factors in slot fs of F, Fc, Fs, and (complex64) the operand-order copies
// Fa, Fw (identical strips share a slot)
hipError_t launch_strip_solve(const DevTables& t, const Geom& g, const Chunks& ch, int s, int fs,
                              const cplx<T>* F, const cplx<T>* Fc, const cplx<T>* Fs, const cplx<T>* Fa,
                              const cplx<T>* Fw, cplx<T>* Yw, int nrhs, const IOSpec& io, hipStream_t st,
                              KTimer* kt = nullptr);

hipError_t launch_apply_A(const DevTables& t, const Geom& g, int nrhs, const double2* u,
                          const double2* f, double2* out, hipStream_t st);
// f - A u (or A u when f is null) on npairs pairs of adjacent columns: cols[2q + 1] == cols[2q] + 1
hipError_t launch_apply_A_pairs(const DevTables& t, const Geom& g, int nrhs, const int* cols,
                               int npairs, const double2* u, const double2* f, double2* out,
                               hipStream_t st);
// Reduced-form stencils on interface windows (u, g window fields; psi, out reduced vectors
// [nrhs][Nrow][2(J-1)] holding columns beta_j, beta_j + 1):
//   mode 0: g = psi - A u on the window columns beta_j - 1, beta_j (psi is 0 on beta_j - 1)
//   mode 1: out = psi - (g - A u) on beta_j, beta_j + 1
//   mode 2: out = A (u + psi - g) on beta_j - 1, beta_j (psi, g: window fields too; the
//           concurrent sweep's v, w' and z)
//   mode 3: g = psi - A u on beta_j - 1, beta_j with psi a full field
//   mode 4: out = g - A u on beta_j, beta_j + 1 (g = 0 on beta_j + 1)
hipError_t launch_stencil_win(int mode, const DevTables& t, const Geom& g, int nrhs, const double2* u,
                              const double2* psi, double2* gw, double2* out, hipStream_t st);

// Batched FP64 vector kernels for GMRES; vectors are [nrhs][n] complex, a basis is
// kmax contiguous vectors of nrhs*n each.
hipError_t launch_dots(const double2* V, int nvec, const double2* w, int nrhs, long n,
                       double2* partial, int nblk, double2* out, hipStream_t st);
hipError_t launch_update(const double2* V, int nvec, const double2* h, double2* w, int nrhs,
                         long n, hipStream_t st);
hipError_t launch_norms(const double2* w, int nrhs, long n, double* partial, int nblk,
                        double* out, hipStream_t st);
hipError_t launch_scale(const double2* w, const double* nrm, double2* out, int nrhs, long n,
                        hipStream_t st);
hipError_t launch_lincomb(const double2* V, int nvec, const double2* y, double2* out,
                          int nrhs, long n, int accumulate, hipStream_t st);
hipError_t launch_gather_cols(const double2* field, const int* cols, int ncols, int nrhs,
                              int Ny, int Nx, double2* red, hipStream_t st);
// field[.., cols[k]] = red[.., k] (add: +=)
hipError_t launch_scatter_cols(const double2* red, const int* cols, int ncols, int nrhs,
                               int Ny, int Nx, double2* field, hipStream_t st, bool add = false);
// zero entries c0 .. c0 + n - 1 of each row of a window field ([nrows][wrow])
hipError_t launch_clear_win_cols(double2* win, long nrows, long wrow, int c0, int n, hipStream_t st);
// zero column cols[k] + shift of every row, k < ncols
// out = x + y + z; x or z may be null
hipError_t launch_sum3(const double2* x, const double2* y, const double2* z, double2* out, long n,
                       hipStream_t st);
// Robin data of a neighbour field: out[r][row] = (vo - rho[row] vi)[r][row] / h^2
hipError_t launch_robin_data(const double2* vo, const double2* vi, const double2* rho, double2* out, int nrhs,
                             long Nrow, double ih2, hipStream_t st);
// out = x + y - z (all non-null)
hipError_t launch_sum_diff(const double2* x, const double2* y, const double2* z, double2* out, long n,
                           hipStream_t st);
int dots_blocks(long n);

// one plane l of the 3-D slab factorisation for every slab: S = T_l - c_l b_{l-1} Gprev,
// inverted in place by blocked Gauss-Jordan; the inverse goes to G64 (FP64, may be null)
// and to out + s * out_stride (complex64 if out_single, else complex128)
hipError_t launch_factor3_plane(const Fac3Args& a, int l, const double2* Gprev, double2* S,
                                double2* Tm, double2* Cm, int* perm, int* pi, int* err,
                                double2* G64, void* out, bool out_single, size_t out_stride,
                                hipStream_t st);
size_t factor3_panel_width();
// complex64 slab factorisation (mixed precision): blocked Gauss-Jordan in place in the
// stored factor F ([slab][plane][Bp*Bp], slab stride `stride`), one plane of the slabs
// s0 .. s0 + ns - 1 per call (disjoint slab sets may run on different streams)
size_t factor3_f32_work_bytes(int J, int Bp);
// stored complex64 slab inverses (J slots of Ny planes, slot stride `stride`) rewritten,
// plane by plane, from column-major into the 16-row panels the sweeps read; work holds
// J Bp^2 complex64 entries
hipError_t launch_factor3_panelize(float2* F, size_t stride, int J, int Ny, int Bp, float2* work, hipStream_t st);
hipError_t launch_factor3_plane_f32(const Fac3Args& a, int l, float2* F, size_t stride, void* work, int* err,
                                    hipStream_t st, int s0, int ns);
template <typename T>
hipError_t launch_strip_solve3(const Solve3Args<T>& a, hipStream_t st, KTimer* kt);

// ---- host core (helm_api.hip) shared with other entry points
// bytes of strip-solver workspace one strip solve of nrhs right-hand sides needs
size_t strip_workspace_bytes(helm_t H, int nrhs);
// helm_strip_solve with the workspace ws (>= strip_workspace_bytes; null: the handle's own)
helm_status strip_solve_into(helm_t H, int strip, int nrhs, const void* r, void* x, void* ws);
hipStream_t handle_stream(helm_t H);
int handle_device(helm_t H);
bool handle_factored(helm_t H);
int handle_strips(helm_t H);
helm_status handle_fail(helm_t H, helm_status code, const std::string& msg);

// ---- misfit and adjoint gradient (kernels_grad.hip)
hipError_t launch_rec_residual(const double2* u, long field, const long* rec, int nrec,
                               const double2* d, int nsrc, double2* r, hipStream_t st);
hipError_t launch_half_sumsq(const double2* r, long n, double* out, hipStream_t st);
hipError_t launch_adjoint_rhs(const double2* r, int nrec, int nsrc, const long* upt, const int* ustart,
                              const int* uidx, int nu, const DevTables& t, const Geom& g, double2* Q,
                              hipStream_t st);
hipError_t launch_grad_m(const double2* u, const double2* z, int nsrc, const DevTables& t,
                         const Geom& g, double* grad, hipStream_t st);

}  // namespace helm

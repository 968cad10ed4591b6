// Internal interface between the C ABI layer (pv_api.cpp) and the HIP kernels
// (pv_kernels.hip).  Not installed; not part of the public ABI.
#pragma once

#ifndef PV_RTC
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#else
// run-time compiled kernels: the fixed-width integers of the RTC runtime header
using __hip_internal::int64_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
#endif

namespace pv {

constexpr int PV_MAX_NB_K = 64;
constexpr int PV_MAX_TERMS_K = 26;   // neighbour offsets per stencil (the C ABI's limit)
// Largest site (n_orb * nb elements) the staged sweep kernel takes; wider
// blocks use the direct kernel.
constexpr int STAGED_MAX_SITE = 128;
// Most slots (per-lane block entries kept in registers) a compiled pattern has.
constexpr int MAX_SLOTS_K = 96;

// Kernel families: a family fixes the stencil's offsets and the zero / real /
// imaginary structure of every block at compile time; values stay runtime.
enum Family : int {
    FAM_GENERIC = 0,     // any offsets in {-1,0,1}^3, dense complex blocks
    FAM_TI = 1,          // 3D TI (Sec. 2.2), n_orb = 4, offsets +-x, +-y, +-z
    FAM_GRAPHENE2 = 2,   // two-site honeycomb, n_orb = 2, offsets +-x, +-y (2D)
    FAM_GRAPHENE4 = 3,   // four-site graphene cell (Sec. 2.1), n_orb = 4 (2D)
    FAM_WEYL = 4,        // Weyl semimetal (Sec. 2.3), n_orb = 2, 3D
    FAM_CODEGEN = 5,     // a stencil's own pattern, generated and compiled at run time
};

// Block-entry codes.
enum : unsigned char { CZ = 0, CR = 1, CI = 2, CC = 3 };

// Epilogue flags of a sweep.
enum : unsigned {
    EP_STORE_Y = 1u,     // write y
    EP_ACC_INIT = 2u,    // acc_out = eta0 * x + eta * y
    EP_ACC_ADD = 4u,     // acc_out = acc_in + eta * y
    EP_DOTS = 8u,        // per-block partial dots (xx, Re xy, Im xy, yy)
    EP_GTERMS = 16u,     // y += sum_j gcoef[j][c] gw_j (adjoint source terms)
    EP_GRAD = 32u,       // grad += gx Re(conj(x) gw_1) + gy Re(conj(y) gw_0) per site/row
    EP_NO_Z = 64u,       // launch-internal: gamma = 0, z is neither loaded nor staged
};

#ifndef PV_RTC
struct SweepParams {
    int family;
    int dtype;            // 0 = complex128, 1 = complex64
    int vtype;            // 0 = float64 field, 1 = float32 field
    int n_orb;
    int n_terms;          // generic family only
    int pot_mode;         // 0 none, 1 site, 2 orbital
    int64_t L[3];
    int periodic[3];
    int nb;
    const void* x;
    const void* z;        // may alias y; NULL if gamma == 0 for all columns
    void* y;
    const void* acc_in;
    void* acc_out;
    const void* V;        // stored field (field == 1)
    int field;            // 0 none, 1 stored array V, 2 counter-based generator
    uint64_t rng_seed;    // field == 2: V[i] = rng_W (u_i - 1/2), u_i from SplitMix64 output i + 1
    double rng_W;
    const void* gw[3];    // adjoint terms (EP_GTERMS / EP_GRAD)
    const double* gcoef;  // device [3][nb] complex
    double* grad;         // device gradient, n_sites (grad_mode 1) or n_rows (grad_mode 2)
    double gx, gy;
    int grad_mode;
    const double* coef;   // device: [(n_terms + 1)][n_orb][n_orb][2], onsite last
    const int* offs;      // device (generic family only): [n_terms][3] offsets, then the
                          // nonzero entries of every block row (row starts, columns)
    const double* colp;   // device: [nb][3] per-column alpha, beta, gamma or NULL
    const void* zero_row;   // device zeros, >= L[0]*n_orb*nb elements
    int slab_rows;          // rows per y-slab of the sweep order (direct kernel)
    int tpb;                // tiles per workgroup (direct kernel; 0 = heuristic)
    int kernel;             // 0 = choose, 1 = direct, 2 = staged
    int generic_stageable;  // generic family: no offset has both a y and a z step
    int generic_side_halo;  // generic family: some offset has both a y and an x step
    int st_E, st_C, st_Bm, st_G8;   // staged kernel: elements per lane, planes per walk,
                                    // strip height, workgroups per XCD (0 = heuristic)
    int st_nt;                      // staged kernel: lanes per workgroup (0 = 256, or 512)
    // launch shape of series steps (EP_ACC_ADD) when acc_kernel > 0, else
    // the fields above
    int acc_kernel, acc_E, acc_C, acc_Bm, acc_G8, acc_nt;
    double alpha, beta, gamma;
    double eta_re, eta_im, eta0_re, eta0_im;
    unsigned ep;
    double* partials;     // [grid][nb][4] when EP_DOTS
    int grid;             // set by launch_sweep: number of workgroups
    // reduction of the previous sweep's partials (red_grid rows) into
    // red_out, by the first wave of workgroup 0 before its tiles (modes of
    // launch_reduce_dots); NULL red_src: none
    const double* red_src;
    double* red_out;
    int red_grid, red_mode, red_M, red_step;
    double red_invD;
    // generated kernels (generic stencils): source of the stencil's pattern
    // struct pv::PatCG, NULL for the interpreted generic kernels; its
    // lattice dimension and side-row flags (x halo, rows at w -+ 1)
    const char* cg_src;
    int cg_dim, cg_halo, cg_sidew;   // cg_sidew: some offset has a y and a z step
    int cg_nocompile;   // take a generated kernel only if loaded (else the interpreted one)
};

// Number of workgroups a sweep of an nb-wide block over the lattice uses
// (partial-dot buffers are sized with it); launch_sweep stores the same
// number in p.grid.
int64_t sweep_grid_max(const int64_t L[3], int n_orb, int nb);
hipError_t launch_sweep(SweepParams& p, int num_cus, hipStream_t s);
// Sweep of a generic stencil with kernels generated from its pattern
// (p.cg_src) and compiled at run time on first use (pv_codegen.cpp).  A
// failed compilation returns hipErrorInvalidImage and leaves the compiler's
// message in codegen_error() (this thread); with p.cg_nocompile an instance
// not loaded yet returns hipErrorNotReady without compiling.
hipError_t launch_codegen(SweepParams& p, int num_cus, hipStream_t s);
const char* codegen_error();
void codegen_clear_error();
// Generated kernel instances loaded in this process (all devices).
int codegen_instances();
// Batched sweeps of a batch whose instances share one generated pattern
// (p.cg_src of any instance): records, launches and compiling the launch's
// instance ahead of a graph capture.
hipError_t codegen_batch_fill_record(const SweepParams& p, int staged, void* dst, int* nblocks);
hipError_t launch_batch_codegen(const SweepParams& p, int staged, const void* table, const int* block_inst,
                                const int* inst_block0, int grid, int red_step, hipStream_t s);
hipError_t codegen_prepare_batch(const SweepParams& p, int staged);

// Fixed-order reduction of [grid][nb][4] partials.
//   mode 0: dots[c][0..3] = sums
//   mode 1: KPM first step: mu[c][0] = xx/D, mu[c][1] = Re xy / D
//   mode 2: KPM step n >= 1: mu[c][2n] = 2 xx/D - mu[c][0], mu[c][2n+1] = 2 Re xy/D - mu[c][1]
hipError_t launch_reduce_dots(const double* partials, int grid, int nb, int mode, double* out,
                              int M, int step, double inv_D, hipStream_t s);

hipError_t launch_scale_block(int dtype, int64_t n_elem, const void* x, double re, double im,
                              void* y, hipStream_t s);

hipError_t launch_gram(int dtype, int64_t rows, int nx, int ny, const void* X, const void* Y,
                       double* partials, int grid, double* G, hipStream_t s);
int gram_grid(int64_t rows, int num_cus);
// Gram and rotation of a search space stored as nblk blocks of bw columns
// (block i at base + i * stride elements): G = A^H B as a dense
// (nblk bw)^2 complex FP64 matrix in one pass; OUT_j = sum_i IN_i Q_ij.
// Partials: nblk^2 * groups * bw^2 * 2 doubles.
int block_gram_groups(int64_t rows, int nblk, int num_cus);
// Source-term table of the KPM adjoint from the moments' cotangent gbar
// [nb][M] (device): table [(M/2 + 1)][3][nb] complex.
hipError_t launch_kpm_adjoint_table(const double* gbar, int nb, int M, double invD, double* table, hipStream_t s);
hipError_t launch_block_gram(int dtype, int64_t rows, int bw, int nblk, const void* A, const void* B,
                             int64_t stride, int hermitian, double* partials, int groups, double* G, hipStream_t s);
hipError_t launch_block_rotate(int dtype, int64_t rows, int bw, int nin, int nout, const void* IN, int64_t in_stride,
                               const double* Q, void* OUT, int64_t out_stride, hipStream_t s);
hipError_t launch_rotate(int dtype, int64_t rows, int nx, int ny, const void* X, const double* Q,
                         int accumulate, void* Y, hipStream_t s);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
hipError_t launch_triad(const void* x, const void* z, void* y, size_t bytes, hipStream_t s);
// workgroups of the read probe (its sink holds one 32-bit word per wave)
constexpr int STREAM_READ_GROUPS = 4096;
hipError_t launch_read(const void* src, size_t bytes, void* sink, hipStream_t s);

// dst[r][dst_col + c] = (re + i im) * src[r][src_col + c] for r < rows,
// c < ncols, blocks of widths src_ld and dst_ld (columns moved between
// blocks, scaled).
hipError_t launch_column_copy(int dtype, int64_t rows, int ncols, const void* src, int src_ld, int src_col,
                              void* dst, int dst_ld, int dst_col, double re, double im, hipStream_t s);

// Bloch start columns: out[s][o][c] = exp(i k_c . r_s) for o == orb[c] on
// the sites of the layer (axis < 0: all sites), else 0.
struct BlochCols {
    double k[64][3];
    int orb[64];
};
hipError_t launch_bloch(int dtype, int64_t n_sites, int n_orb, int nb, int Lx, int Ly, const BlochCols& cols,
                        int axis, int64_t index, void* out, hipStream_t s);

// Random start blocks: out[e] for e < n takes the counter-based generator's
// output number i0 + e + 1 of the stream seeded with seed, mapped to a
// random phase (kind 0) or a Z4 phase (kind 1).
hipError_t launch_random_block(int dtype, int kind, int64_t n, uint64_t seed, uint64_t i0, void* out, hipStream_t s);

// Batched sweeps: one argument record per instance (built on the host with
// batch_fill_record from that instance's launch description), a table of
// records in device memory, and per-workgroup instance maps.  staged: every
// instance takes the staged kernel (compiled family, 16-byte aligned blocks;
// then *nblocks is a multiple of 8 and instances must start at multiples of
// 8), else the direct kernel over the whole lattice.  *nblocks receives the
// instance's workgroup count.  launch_batch_sweep takes the launch
// description of any instance (family, types, nb, tuning, epilogue).
size_t batch_record_bytes();
// dst = 0 (bytes a multiple of 4)
hipError_t launch_zero(void* dst, size_t bytes, hipStream_t s);
hipError_t batch_fill_record(const SweepParams& p, int staged, void* dst, int* nblocks);
// red_step: the moment step the records' folded reductions write (their
// red_* fields say what to reduce; see SweepParams)
hipError_t launch_batch_sweep(const SweepParams& p, int staged, const void* table, const int* block_inst,
                              const int* inst_block0, int grid, int red_step, hipStream_t s);
hipError_t launch_batch_reduce(const double* partials, const int* inst_block0, int n_inst, int nb, int mode,
                               double* mu, int M, int step, const double* invD, hipStream_t s);

#endif  // PV_RTC
}  // namespace pv

namespace pv {

// ---------------------------------------------------------------------------
// Compiled stencil families.  Offsets use the descriptor convention
// (H x)[s] += B_t x[s + d_t]; code[t][o][o'] says which entries of B_t may be
// nonzero and whether they are real (CR), imaginary (CI) or complex (CC).
// Row NT of `code` is the on-site block (its diagonal also carries V - beta).
// ---------------------------------------------------------------------------

// 3D TI (Sec. 2.2) with Gamma^1 = tau_z sigma_0, Gamma^{j+1} = tau_x sigma_j:
// B_{-e_j} = -(t/2)(G1 - i G_{j+1}), B_{+e_j} = B_{-e_j}^H, E0 = m G1.
struct PatTI {
    static constexpr int FAMILY = FAM_TI, NO = 4, NT = 6, DIM = 3;
    static constexpr bool SIDE_HALO = false, SIDE_W = false;
    static constexpr int off[NT][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
    static constexpr unsigned char code[NT + 1][NO][NO] = {
        {{CR, CZ, CZ, CI}, {CZ, CR, CI, CZ}, {CZ, CI, CR, CZ}, {CI, CZ, CZ, CR}},
        {{CR, CZ, CZ, CI}, {CZ, CR, CI, CZ}, {CZ, CI, CR, CZ}, {CI, CZ, CZ, CR}},
        {{CR, CZ, CZ, CR}, {CZ, CR, CR, CZ}, {CZ, CR, CR, CZ}, {CR, CZ, CZ, CR}},
        {{CR, CZ, CZ, CR}, {CZ, CR, CR, CZ}, {CZ, CR, CR, CZ}, {CR, CZ, CZ, CR}},
        {{CR, CZ, CI, CZ}, {CZ, CR, CZ, CI}, {CI, CZ, CR, CZ}, {CZ, CI, CZ, CR}},
        {{CR, CZ, CI, CZ}, {CZ, CR, CZ, CI}, {CI, CZ, CR, CZ}, {CZ, CI, CZ, CR}},
        {{CR, CZ, CZ, CZ}, {CZ, CR, CZ, CZ}, {CZ, CZ, CR, CZ}, {CZ, CZ, CZ, CR}},
    };
};

// Two-site honeycomb on an (i, j) grid: A(s) <- B(s), B(s - e_i), B(s - e_j).
struct PatGraphene2 {
    static constexpr int FAMILY = FAM_GRAPHENE2, NO = 2, NT = 4, DIM = 2;
    static constexpr bool SIDE_HALO = false, SIDE_W = false;
    static constexpr int off[NT][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}};
    static constexpr unsigned char code[NT + 1][NO][NO] = {
        {{CZ, CR}, {CZ, CZ}}, {{CZ, CZ}, {CR, CZ}},
        {{CZ, CR}, {CZ, CZ}}, {{CZ, CZ}, {CR, CZ}},
        {{CZ, CR}, {CR, CZ}},
    };
};

// Four-site graphene cell (Sec. 2.1): B_{-x} = T_x, B_{+x} = T_x^T,
// B_{-y} = T_y, B_{+y} = T_y^T, E0 = T_n (chain 0-1-2-3).
struct PatGraphene4 {
    static constexpr int FAMILY = FAM_GRAPHENE4, NO = 4, NT = 4, DIM = 2;
    static constexpr bool SIDE_HALO = false, SIDE_W = false;
    static constexpr int off[NT][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}};
    static constexpr unsigned char code[NT + 1][NO][NO] = {
        {{CZ, CZ, CZ, CZ}, {CR, CZ, CZ, CZ}, {CZ, CZ, CZ, CR}, {CZ, CZ, CZ, CZ}},
        {{CZ, CR, CZ, CZ}, {CZ, CZ, CZ, CZ}, {CZ, CZ, CZ, CZ}, {CZ, CZ, CR, CZ}},
        {{CZ, CZ, CZ, CR}, {CZ, CZ, CZ, CZ}, {CZ, CZ, CZ, CZ}, {CZ, CZ, CZ, CZ}},
        {{CZ, CZ, CZ, CZ}, {CZ, CZ, CZ, CZ}, {CZ, CZ, CZ, CZ}, {CR, CZ, CZ, CZ}},
        {{CZ, CR, CZ, CZ}, {CR, CZ, CR, CZ}, {CZ, CR, CZ, CR}, {CZ, CZ, CR, CZ}},
    };
};

// Weyl semimetal (Sec. 2.3): B_{+-x} = sigma_x/2, B_{-y} = (sigma_x + i sigma_y)/2,
// B_{-z} = (sigma_x + i sigma_z)/2 (and their adjoints), E0 = -sigma_x(2 + cos k0).
struct PatWeyl {
    static constexpr int FAMILY = FAM_WEYL, NO = 2, NT = 6, DIM = 3;
    static constexpr bool SIDE_HALO = false, SIDE_W = false;
    static constexpr int off[NT][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
    static constexpr unsigned char code[NT + 1][NO][NO] = {
        {{CZ, CR}, {CR, CZ}}, {{CZ, CR}, {CR, CZ}},
        {{CZ, CR}, {CZ, CZ}}, {{CZ, CZ}, {CR, CZ}},
        {{CI, CR}, {CR, CI}}, {{CI, CR}, {CR, CI}},
        {{CZ, CR}, {CR, CZ}},
    };
};

}  // namespace pv

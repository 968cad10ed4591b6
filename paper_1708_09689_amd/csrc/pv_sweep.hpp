#pragma once
// HIP sweep kernels for gfx950 (MI355X) and their launchers, as templates
// over the stencil family: the matrix-free stencil sweep with fused
// Chebyshev epilogues and partial dot products.  Each family is compiled in
// a translation unit of its own (pv_fam_*.hip), so the families build in
// parallel; internal to the library, every includer gets its own copies.
//
// The sweep evaluates, per column c of an nb-wide block (Sec. 3.2, generated
// spMVM listing, with scale_h = alpha, shift_h = beta, scale_z = gamma):
//     y = alpha (H x - beta x) + gamma z
// where H acts matrix-free through the stencil blocks of the lattice
// (Sec. 3.2 DSL: one block per neighbour offset), and optionally
//     acc = eta0 x + eta y   or   acc += eta y     (Chebyshev series, Sec. 4)
//     partial sums of <x,x>, <x,y>, <y,y>           (fused dots, Sec. 3.2/3.5)
//
// Work decomposition: one lane owns one element (site s, orbital row o,
// column c) of the output block.  A workgroup of 256 lanes covers 256
// consecutive elements, so every load of a neighbour's entries is a fully
// coalesced wave-wide access of 64 consecutive complex numbers (shifted by
// the neighbour's site offset; entries of other orbitals of the same site
// are a fixed lane-dependent offset within the same cache lines).  Because
// n_orb * nb divides 256, a lane keeps the same (o, c) for the whole launch:
// its row's stencil coefficients live in registers.  Block structure is
// compiled in per family: for every neighbour block and entry kind (real,
// imaginary, complex) the kernel carries "slots" -- the k-th nonzero of that
// kind in the lane's row -- so the TI stencil costs 12 two-FMA complex
// updates per row.  The grid is persistent, sized from the occupancy of the
// instantiation, and XCD-aware: workgroup b runs on XCD b % 8, each XCD takes
// one contiguous eighth of the tiles, and its resident workgroups sweep that
// range together, so the +-y / +-z neighbour rows they read were fetched by
// the same XCD shortly before (same L2).
#include "pv_kernels.hpp"

#ifndef PV_RTC
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <utility>
#endif

namespace pv {
namespace {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
    T re, im;
};

template <int V>
struct IntC {
    static constexpr int value = V;
};

template <int N, int I = 0, typename F>
__device__ __forceinline__ void sfor(F&& f) {
    if constexpr (I < N) {
        f(IntC<I>{});
        sfor<N, I + 1>(f);
    }
}

constexpr int kBlock = 256;

template <typename T>
using vec2 = T __attribute__((ext_vector_type(2)));
using u32x4 = unsigned int __attribute__((ext_vector_type(4)));

// Round-up division by a runtime constant (Granlund & Montgomery): exact for
// every 32-bit numerator.
struct FastDiv {
    uint32_t d, m, l;
};

inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f{d, 0u, 0u};
    if (d > 1) {
        uint32_t l = 0;
        while ((1ull << l) < d) ++l;
        f.l = l;
        f.m = uint32_t((((1ull << 32) * ((1ull << l) - d)) / d) + 1);
    }
    return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
    if (f.d == 1) return n;
    const uint32_t t = __umulhi(n, f.m);
    return (t + ((n - t) >> 1)) >> (f.l - 1);
}

template <typename T, typename VT>
struct KArgs {
    const cplx<T>* x;
    const cplx<T>* z;
    cplx<T>* y;
    const cplx<T>* acc_in;
    cplx<T>* acc_out;
    const cplx<T>* zsrc;    // z, or x when no column reads z (a valid dummy)
    const cplx<T>* asrc;    // acc_in, or x when not accumulating
    const VT* V;
    int field;              // 0 none, 1 stored array V, 2 counter-based generator
    uint64_t rng_seed;
    double rng_W;
    const cplx<T>* gw0;     // adjoint terms: w_{k-1}, w_k, w_{k+1} (or NULL)
    const cplx<T>* gw1;
    const cplx<T>* gw2;
    const double* gcoef;    // [3][nb] complex coefficients of the gw terms
    double* grad;           // on-site field gradient
    double gx, gy;
    int ggroup;             // lanes per gradient entry: n_orb*nb (site field) or nb (orbital field)
    const double* coef;
    const int* offs;
    const double* colp;
    double* partials;
    const double* red_src;   // previous sweep's partials reduced at the start (or NULL)
    double* red_out;
    int red_grid, red_mode, red_M, red_step;
    double red_invD;
    int64_t n_elem, ntiles;
    int tpb;
    // traversal: XCD part k (rows y in [Ly k/8, Ly (k+1)/8), all z) is swept
    // in slabs of BY rows, each slab plane by plane, each plane row by row
    const cplx<T>* zero_row;   // rowel zeros: neighbour rows dropped by open BCs read here
    int rowel, ntx, BY;
    FastDiv fd_ntx, fd_slab, fd_pf;
    int Lx, Ly, Lz;
    int px, py, pz;
    int nb, lognb, logsite;
    int n_terms, pot_mode;
    double alpha, beta, gamma;
    double eta_re, eta_im, eta0_re, eta0_im;
    unsigned ep;
    // staged traversal (staged_kernel): column tiles of one row walked along
    // the outer dimension w; m is the middle dimension (y in 3D, none in 2D)
    int st_site, st_seg, st_nxs;   // elements per site, ring row length, column tiles per row
    int st_Lm, st_Lw, st_pm, st_pw;
    int st_C, st_Bm, st_parts;     // planes per walk, strip height, 8 XCD parts or 1
};

template <typename T>
__device__ __forceinline__ void mac(T& ar, T& ai, unsigned char k, T cr, T ci, cplx<T> v) {
    if (k == CR) { ar += cr * v.re; ai += cr * v.im; }
    else if (k == CI) { ar -= ci * v.im; ai += ci * v.re; }
    else if (k == CC) { ar += cr * v.re - ci * v.im; ai += cr * v.im + ci * v.re; }
}

// Counter-based generator of the on-the-fly field (SplitMix64, Steele, Lea
// and Flood 2014): output i + 1 of the stream seeded with `seed`, i.e. the
// mixing function applied to seed + (i + 1) * golden gamma.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// On-site field value at index i (site, or orbital row for per-orbital
// fields): the stored array, or W (u - 1/2) with u the generator's top 53
// bits times 2^-53 -- u - 1/2 is exact, so the value is one rounded product.
template <typename T, typename VT>
__device__ __forceinline__ T field_at(const KArgs<T, VT>& a, int64_t i) {
    if (a.field == 2) {
        const double u = double(splitmix64_at(a.rng_seed, uint64_t(i)) >> 11) * 0x1.0p-53;
        return T(a.rng_W * (u - 0.5));
    }
    return T(a.V[i]);
}

// Slots of a compiled family: for block t (t == NT: off-diagonal part of the
// on-site block) and entry kind, slot k holds the k-th nonzero of that kind
// in each row o (q[o] = its column, -1 if the row has fewer).
template <class P>
struct Slots {
    static constexpr int MAX = MAX_SLOTS_K;
    int n = 0;
    int t[MAX] = {};
    unsigned char kind[MAX] = {};
    signed char q[MAX][4] = {};
    bool same[MAX] = {};   // every row's entry sits in its own orbital (orbital offset 0)
    constexpr Slots() {
        constexpr int NO = P::NO;
        for (int tt = 0; tt <= P::NT; ++tt)
            for (int kd = 1; kd <= 3; ++kd) {
                int K = 0;
                for (int o = 0; o < NO; ++o) {
                    int cnt = 0;
                    for (int qq = 0; qq < NO; ++qq)
                        if (!(tt == P::NT && qq == o) && P::code[tt][o][qq] == kd) ++cnt;
                    if (cnt > K) K = cnt;
                }
                for (int k = 0; k < K; ++k) {
                    t[n] = tt;
                    kind[n] = (unsigned char)kd;
                    for (int o = 0; o < 4; ++o) q[n][o] = -1;
                    for (int o = 0; o < NO; ++o) {
                        int cnt = 0;
                        for (int qq = 0; qq < NO; ++qq)
                            if (!(tt == P::NT && qq == o) && P::code[tt][o][qq] == kd) {
                                if (cnt == k) q[n][o] = (signed char)qq;
                                ++cnt;
                            }
                    }
                    same[n] = true;
                    for (int o = 0; o < NO; ++o)
                        if (q[n][o] >= 0 && q[n][o] != o) same[n] = false;
                    ++n;
                }
            }
    }
};

// Generic family descriptor: NO orbitals, runtime offsets, dense blocks.
// SH (every pattern's SIDE_HALO): the staged kernel loads the side rows with
// the x halo (stencils with hops that have a y and an x step).
template <int NO_, bool SH = false>
struct PatGeneric {
    static constexpr int FAMILY = FAM_GENERIC, NO = NO_, NT = 0, DIM = 3;
    static constexpr bool SIDE_HALO = SH, SIDE_W = false;
    static constexpr int off[1][3] = {{0, 0, 0}};
    static constexpr unsigned char code[1][NO_][NO_] = {};   // no compiled slots
};

template <class P>
constexpr bool side_halo() {
    return P::SIDE_HALO;
}

template <typename T>
__device__ __forceinline__ cplx<T> ld_nt(const cplx<T>* p) {
    const vec2<T> v = __builtin_nontemporal_load(reinterpret_cast<const vec2<T>*>(p));
    return cplx<T>{v.x, v.y};
}

template <typename T>
__device__ __forceinline__ void st_nt(cplx<T>* p, T re, T im) {
    vec2<T> v;
    v.x = re;
    v.y = im;
    __builtin_nontemporal_store(v, reinterpret_cast<vec2<T>*>(p));
}

// Loads at a 32-bit byte offset from a (workgroup-uniform) row pointer.
template <typename T>
__device__ __forceinline__ cplx<T> ld_row(const cplx<T>* row, uint32_t boff) {
    return *reinterpret_cast<const cplx<T>*>(reinterpret_cast<const char*>(row) + boff);
}

template <typename T>
__device__ __forceinline__ cplx<T> ld_row_nt(const cplx<T>* row, uint32_t boff) {
    return ld_nt(reinterpret_cast<const cplx<T>*>(reinterpret_cast<const char*>(row) + boff));
}

// Epilogue shared by every family: y = alpha h + gamma z (+ sum_j g_j w_j),
// store / accumulate, FP64 partial dots of (x, y), and the on-site field
// gradient.  zv and av were loaded at the top of the element
// (unconditionally, from a valid address) so that every load of an element
// is in flight at the same time; gamma == 0 selects zero instead of
// gamma * z, so z is never used for such columns.
//
// Adjoint options (Clenshaw-type recurrences for gradients):
//   EP_GTERMS  y += sum_{j=0..2} gcoef[j][c] * gw_j[e]   (complex coefficients;
//              gw_j == NULL skips the term)
//   EP_GRAD    grad[site or row] += gx Re(conj(x) gw_1) + gy Re(conj(y) gw_0),
//              summed over the site's (or row's) lanes with a fixed xor tree
//              and written by one lane, read-modify-write (no atomics)
template <typename T, typename VT>
__device__ __forceinline__ void epilogue_ep(const KArgs<T, VT>& a, const unsigned ep, int64_t e, int64_t gidx,
                                            int glane, cplx<T> xc, cplx<T> zv, cplx<T> av, T hr, T hi, T alT, T gaT,
                                            T er, T ei, T e0r, T e0i, int c, double& dxx, double& dxr, double& dxi,
                                            double& dyy) {
    T yr = alT * hr, yi = alT * hi;
    yr += (gaT != T(0)) ? gaT * zv.re : T(0);
    yi += (gaT != T(0)) ? gaT * zv.im : T(0);
    cplx<T> gv[3] = {{T(0), T(0)}, {T(0), T(0)}, {T(0), T(0)}};
    if (ep & (EP_GTERMS | EP_GRAD)) {
        const cplx<T>* gws[3] = {a.gw0, a.gw1, a.gw2};
        for (int j = 0; j < 3; ++j)
            if (gws[j] != nullptr) gv[j] = ld_nt(gws[j] + e);
    }
    if (ep & EP_GTERMS) {
        for (int j = 0; j < 3; ++j) {
            const T cr = T(a.gcoef[(j * a.nb + c) * 2]), ci = T(a.gcoef[(j * a.nb + c) * 2 + 1]);
            yr += cr * gv[j].re - ci * gv[j].im;
            yi += cr * gv[j].im + ci * gv[j].re;
        }
    }
    if (ep & EP_STORE_Y) st_nt(a.y + e, yr, yi);
    if (ep & EP_ACC_INIT) {
        st_nt(a.acc_out + e, e0r * xc.re - e0i * xc.im + er * yr - ei * yi,
              e0r * xc.im + e0i * xc.re + er * yi + ei * yr);
    } else if (ep & EP_ACC_ADD) {
        st_nt(a.acc_out + e, av.re + er * yr - ei * yi, av.im + er * yi + ei * yr);
    }
    if (ep & EP_DOTS) {
        const double xr = double(xc.re), xi = double(xc.im);
        const double dyr = double(yr), dyi = double(yi);
        dxx += xr * xr + xi * xi;
        dxr += xr * dyr + xi * dyi;
        dxi += xr * dyi - xi * dyr;
        dyy += dyr * dyr + dyi * dyi;
    }
    if (ep & EP_GRAD) {
        double g = a.gx * (double(xc.re) * double(gv[1].re) + double(xc.im) * double(gv[1].im)) +
                   a.gy * (double(yr) * double(gv[0].re) + double(yi) * double(gv[0].im));
        for (int m = 1; m < a.ggroup; m <<= 1) g += __shfl_xor(g, m);
        if (glane == 0) a.grad[gidx] += g;
    }
}

template <typename T, typename VT>
__device__ __forceinline__ void epilogue(const KArgs<T, VT>& a, int64_t e, int64_t gidx, int glane, cplx<T> xc,
                                         cplx<T> zv, cplx<T> av, T hr, T hi, T alT, T gaT, T er, T ei, T e0r,
                                         T e0i, int c, double& dxx, double& dxr, double& dxi, double& dyy) {
    epilogue_ep(a, a.ep, e, gidx, glane, xc, zv, av, hr, hi, alT, gaT, er, ei, e0r, e0i, c, dxx, dxr, dxi, dyy);
}

template <typename T>
__device__ __forceinline__ cplx<T> zero_unless(bool ok, cplx<T> v) {
    return cplx<T>{ok ? v.re : T(0), ok ? v.im : T(0)};
}

#ifndef PV_SWEEP_WAVES_PER_EU
#define PV_SWEEP_WAVES_PER_EU 1
#endif
#ifndef PV_STAGED_WAVES_PER_EU
#define PV_STAGED_WAVES_PER_EU 2
#endif


// Row (y + dy, z + dz) of row (y, z), wrapped along periodic dimensions;
// false when an open boundary drops it.  Uniform over a tile.
template <typename A>
__device__ __forceinline__ bool neighbour_row(const A& a, int y, int z, int dy, int dz, int& row) {
    int yn = y + dy, zn = z + dz;
    bool ok = true;
    if (dy) {
        const bool lo = yn < 0, hi = yn >= a.Ly;
        ok = ok && (a.py || !(lo || hi));
        yn += lo ? a.Ly : (hi ? -a.Ly : 0);
    }
    if (dz) {
        const bool lo = zn < 0, hi = zn >= a.Lz;
        ok = ok && (a.pz || !(lo || hi));
        zn += lo ? a.Lz : (hi ? -a.Lz : 0);
    }
    row = zn * a.Ly + yn;
    return ok;
}

__device__ __forceinline__ FastDiv make_fastdiv_dev(uint32_t d) {
    FastDiv f{d, 0u, 0u};
    if (d > 1) {
        const uint32_t l = 32u - __clz(d - 1u);
        f.l = l;
        f.m = uint32_t((((1ull << 32) * ((1ull << l) - d)) / d) + 1);
    }
    return f;
}

// Element offset of the x-neighbour (x + dx) inside its row, relative to the
// lane's own element xe; false when an open boundary drops it.
template <typename A>
__device__ __forceinline__ bool x_shift(const A& a, int x, int dx, int& dxe) {
    const int site = 1 << a.logsite;
    if (dx == 0) { dxe = 0; return true; }
    const int xn = x + dx;
    if (xn < 0) { dxe = (a.Lx - 1) * site; return a.px; }
    if (xn >= a.Lx) { dxe = -(a.Lx - 1) * site; return a.px; }
    dxe = dx * site;
    return true;
}

// Per-lane data of a compiled family: for every slot the complex coefficient
// of the lane's row and the element offset of the partner orbital inside the
// site (zero coefficient where the row has fewer entries of that kind).
template <class P, typename T, int NS, int NA>
__device__ __forceinline__ void slot_coefficients(const double* coef, int o, int nb, T (&cre)[NA], T (&cim)[NA],
                                                  int (&dq)[NA]) {
    constexpr int NO = P::NO;
    static constexpr Slots<P> S{};
    sfor<NS>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        int q = S.q[j][0];
        if constexpr (NO > 1) { if (o == 1) q = S.q[j][1]; }
        if constexpr (NO > 2) { if (o == 2) q = S.q[j][2]; if (o == 3) q = S.q[j][3]; }
        if (q >= 0) {
            const double* e = coef + ((S.t[j] * NO + o) * NO + q) * 2;
            cre[j] = T(e[0]);
            cim[j] = T(e[1]);
            dq[j] = (q - o) * nb;
        } else {
            cre[j] = T(0);
            cim[j] = T(0);
            dq[j] = 0;
        }
    });
}

// The work of one workgroup: tiles [t0, t1) of the part of the lattice made of
// rows y in [y0, y0 + ny) (all z), swept slab by slab; partial dots go to
// partials[b_out].
// Fixed-order sum over the partial rows of block column c by one wave
// (lane-strided sums, then an xor tree); lane 0 stores the result: mode 0
// the four dots, mode 1 mu_0 and mu_1 (divided by D), mode 2 the moments
// mu_2step = 2 xx / D - mu_0 and mu_2step+1 = 2 xy / D - mu_1.
__device__ __forceinline__ void reduce_column_wave(const double* __restrict__ partials, int grid, int nb, int c,
                                                  int mode, double* out, int M, int step, double inv_D, int lane) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int b = lane; b < grid; b += 64) {
        const double* q = partials + ((size_t)b * nb + c) * 4;
        s0 += q[0];
        s1 += q[1];
        s2 += q[2];
        s3 += q[3];
    }
    for (int m = 32; m >= 1; m >>= 1) {
        s0 += __shfl_xor(s0, m);
        s1 += __shfl_xor(s1, m);
        s2 += __shfl_xor(s2, m);
        s3 += __shfl_xor(s3, m);
    }
    if (lane == 0) {
        if (mode == 0) {
            out[c * 4 + 0] = s0;
            out[c * 4 + 1] = s1;
            out[c * 4 + 2] = s2;
            out[c * 4 + 3] = s3;
        } else if (mode == 1) {
            out[(size_t)c * M + 0] = s0 * inv_D;
            out[(size_t)c * M + 1] = s1 * inv_D;
        } else {
            double* mu = out + (size_t)c * M;
            mu[2 * step] = 2.0 * s0 * inv_D - mu[0];
            mu[2 * step + 1] = 2.0 * s1 * inv_D - mu[1];
        }
    }
}

// The previous sweep's reduction, folded into this one: the first wave of
// the leading workgroup (workgroup 0, or an instance's first in a batched
// launch) reduces every column before its tiles.  The partials were written
// by the previous launch, so they are complete and visible.
template <typename T, typename VT>
__device__ __forceinline__ void fused_reduction(const KArgs<T, VT>& a, bool lead, int tid) {
    if (a.red_src != nullptr && lead && tid < 64)
        for (int c = 0; c < a.nb; ++c)
            reduce_column_wave(a.red_src, a.red_grid, a.nb, c, a.red_mode, a.red_out, a.red_M, a.red_step,
                               a.red_invD, tid);
}

template <class P, typename T, typename VT>
__device__ __forceinline__ void sweep_block(const KArgs<T, VT>& a, int b_out, int y0, int ny, int64_t t0,
                                            int64_t t1, bool lead) {
    constexpr int NO = P::NO;
    const int tid = threadIdx.x;
    const int nb = a.nb;
    const int c = tid & (nb - 1);
    const int o = (tid >> a.lognb) & (NO - 1);
    fused_reduction(a, lead, tid);

    double al = a.alpha, be = a.beta, ga = a.gamma;
    if (a.colp != nullptr) {
        al = a.colp[3 * c];
        be = a.colp[3 * c + 1];
        ga = a.colp[3 * c + 2];
    }
    const T alT = T(al), beT = T(be), gaT = T(ga);
    const T er = T(a.eta_re), ei = T(a.eta_im), e0r = T(a.eta0_re), e0i = T(a.eta0_im);

    // diagonal of the on-site block for this lane's row
    const int nt_onsite = (P::FAMILY != FAM_GENERIC) ? P::NT : a.n_terms;
    const T dgr = T(a.coef[(((size_t)nt_onsite * NO + o) * NO + o) * 2]);
    const T dgi = T(a.coef[(((size_t)nt_onsite * NO + o) * NO + o) * 2 + 1]);

    double dxx = 0.0, dxr = 0.0, dxi = 0.0, dyy = 0.0;

    // per-lane slot data of compiled families
    static constexpr Slots<P> S{};
    constexpr int NS = (P::FAMILY != FAM_GENERIC) ? S.n : 0;
    T cre[NS > 0 ? NS : 1], cim[NS > 0 ? NS : 1];
    int dq[NS > 0 ? NS : 1];
    slot_coefficients<P, T, NS>(a.coef, o, nb, cre, cim, dq);

    // generic stencils: the nonzero entries of every block row (row starts,
    // columns, values; the host packs them after the offsets and the dense
    // blocks), staged in LDS once per workgroup
    constexpr int GMAX = (PV_MAX_TERMS_K + 1) * NO * NO;
    __shared__ int g_ptr[P::FAMILY == FAM_GENERIC ? (PV_MAX_TERMS_K + 1) * NO + 1 : 1];
    __shared__ int g_col[P::FAMILY == FAM_GENERIC ? GMAX : 1];
    __shared__ cplx<T> g_val[P::FAMILY == FAM_GENERIC ? GMAX : 1];
    if constexpr (P::FAMILY == FAM_GENERIC) {
        const int nptr = (a.n_terms + 1) * NO + 1;
        const int* gp = a.offs + 3 * a.n_terms;
        const int nnz = gp[nptr - 1];
        const double* gv = a.coef + (size_t)(a.n_terms + 1) * NO * NO * 2;
        for (int i = tid; i < nptr; i += kBlock) g_ptr[i] = gp[i];
        for (int i = tid; i < nnz; i += kBlock) {
            g_col[i] = gp[nptr + i];
            g_val[i] = cplx<T>{T(gv[2 * i]), T(gv[2 * i + 1])};
        }
        __syncthreads();
    }

    constexpr uint32_t ES = sizeof(cplx<T>);
    for (int64_t t = t0; t < t1; ++t) {
        // tile -> (row, x-tile): uniform over the workgroup.  Part k is swept
        // in slabs of BY rows; a slab plane by plane (z), a plane row by row.
        const uint32_t tt32 = uint32_t(t);
        const uint32_t slab_tiles = uint32_t(a.ntx) * uint32_t(a.BY) * uint32_t(a.Lz);
        const uint32_t yb = fdiv(tt32, a.fd_slab);
        const uint32_t rr = tt32 - yb * slab_tiles;
        const int by = min(a.BY, ny - int(yb) * a.BY);
        const uint32_t ptiles = uint32_t(a.ntx) * uint32_t(by);
        const uint32_t zz = (by == a.BY) ? fdiv(rr, a.fd_pf) : fdiv(rr, make_fastdiv_dev(ptiles));
        const uint32_t r2 = rr - zz * ptiles;
        const uint32_t yy = fdiv(r2, a.fd_ntx);
        const int xt = int(r2 - yy * uint32_t(a.ntx));
        const int y = y0 + int(yb) * a.BY + int(yy);
        const int z = int(zz);
        const int row = z * a.Ly + y;
        const int xe = xt * kBlock + tid;           // element inside the row
        if (xe >= a.rowel) continue;                // ragged end of the row
        const int x = xe >> a.logsite;
        const int64_t rb = (int64_t)row * a.rowel;
        const uint32_t off0 = uint32_t(xe) * ES;    // byte offset inside a row
        const cplx<T>* xrow = a.x + rb;
        const cplx<T> xc = ld_row(xrow, off0);
        const cplx<T> zv = ld_row_nt(a.zsrc + rb, off0);
        cplx<T> av{T(0), T(0)};
        if (a.ep & EP_ACC_ADD) av = ld_row_nt(a.acc_in + rb, off0);
        T vs = T(0);
        if (a.field != 0) {
            const int64_t vs0 = (int64_t)row * a.Lx * (a.pot_mode == 1 ? 1 : NO);
            vs = field_at(a, a.pot_mode == 1 ? vs0 + x : vs0 + x * NO + o);
        }
        T hr, hi;
        const T d = dgr - beT + vs;
        hr = d * xc.re - dgi * xc.im;
        hi = d * xc.im + dgi * xc.re;
        if constexpr (P::FAMILY != FAM_GENERIC) {
            cplx<T> nv[NS > 0 ? NS : 1];
            bool okt[P::NT > 0 ? P::NT : 1];
            sfor<P::NT>([&](auto tt) {
                constexpr int tb = decltype(tt)::value;
                constexpr int dy = P::off[tb][1], dz = P::off[tb][2];
                const cplx<T>* prow = xrow;
                if constexpr (dy != 0 || dz != 0) {
                    int nrow;
                    const bool rok = neighbour_row(a, y, z, dy, dz, nrow);
                    prow = rok ? a.x + (int64_t)nrow * a.rowel : a.zero_row;
                }
                int dxe;
                okt[tb] = x_shift(a, x, P::off[tb][0], dxe);
                sfor<NS>([&](auto jj) {
                    constexpr int j = decltype(jj)::value;
                    if constexpr (S.t[j] == tb) nv[j] = ld_row(prow, uint32_t(xe + dxe + dq[j]) * ES);
                });
            });
            sfor<NS>([&](auto jj) {
                constexpr int j = decltype(jj)::value;
                if constexpr (S.t[j] == P::NT) nv[j] = ld_row(xrow, uint32_t(xe + dq[j]) * ES);
            });
            sfor<NS>([&](auto jj) {
                constexpr int j = decltype(jj)::value;
                if constexpr (S.t[j] < P::NT && P::off[S.t[j] < P::NT ? S.t[j] : 0][0] != 0) {
                    // x neighbour: lane-dependent open boundary
                    if (!a.px) nv[j] = zero_unless(okt[S.t[j]], nv[j]);
                }
                mac<T>(hr, hi, S.kind[j], cre[j], cim[j], nv[j]);
            });
        } else {
            // nonzero entries only; the loads of a term are issued together
            const int own = xe - o * nb;            // orbital-0 element of this site and column
            for (int tb = 0; tb < a.n_terms; ++tb) {
                const int dy = a.offs[3 * tb + 1], dz = a.offs[3 * tb + 2];
                int nrow;
                const bool rok = neighbour_row(a, y, z, dy, dz, nrow);
                const cplx<T>* prow = rok ? a.x + (int64_t)nrow * a.rowel : a.zero_row;
                int dxe;
                const bool ok = x_shift(a, x, a.offs[3 * tb], dxe);
                const int e0 = g_ptr[tb * NO + o], ne = g_ptr[tb * NO + o + 1] - e0;
                cplx<T> v[NO];
#pragma unroll
                for (int k = 0; k < NO; ++k)
                    if (k < ne) v[k] = ld_row(prow, uint32_t(own + dxe + g_col[e0 + k] * nb) * ES);
#pragma unroll
                for (int k = 0; k < NO; ++k)
                    if (k < ne) mac<T>(hr, hi, CC, g_val[e0 + k].re, g_val[e0 + k].im, zero_unless(ok, v[k]));
            }
            const int e0 = g_ptr[a.n_terms * NO + o], e1 = g_ptr[a.n_terms * NO + o + 1];
            for (int e = e0; e < e1; ++e)
                mac<T>(hr, hi, CC, g_val[e].re, g_val[e].im, ld_row(xrow, uint32_t(own + g_col[e] * nb) * ES));
        }
        const int64_t site = (int64_t)row * a.Lx + x;
        const int64_t gidx = a.ggroup == nb ? site * NO + o : site;
        epilogue(a, rb + xe, gidx, tid & (a.ggroup - 1), xc, zv, av, hr, hi, alT, gaT, er, ei, e0r, e0i, c, dxx, dxr,
                 dxi, dyy);
    }

    if (a.ep & EP_DOTS) {
        // lanes with the same column: lane = (site * NO + o) * nb + c inside the wave
        for (int m = nb; m < 64; m <<= 1) {
            dxx += __shfl_xor(dxx, m);
            dxr += __shfl_xor(dxr, m);
            dxi += __shfl_xor(dxi, m);
            dyy += __shfl_xor(dyy, m);
        }
        __shared__ double red[kBlock / 64][PV_MAX_NB_K][4];
        const int wave = tid >> 6, lane = tid & 63;
        if (lane < nb) {
            red[wave][lane][0] = dxx;
            red[wave][lane][1] = dxr;
            red[wave][lane][2] = dxi;
            red[wave][lane][3] = dyy;
        }
        __syncthreads();
        if (tid < nb * 4) {
            const int cc = tid >> 2, k = tid & 3;
            double sum = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) sum += red[w][cc][k];
            a.partials[((size_t)b_out * nb + cc) * 4 + k] = sum;
        }
    }
}

// One sweep over a whole lattice.  Workgroup b runs on XCD b % 8 (the
// hardware deals workgroups out round-robin); XCD k owns the rows y in
// [Ly k/8, Ly (k+1)/8) for every z and its workgroups sweep them slab by slab,
// so the +-y and +-z neighbour rows a tile reads were fetched into the same L2
// shortly before.
template <class P, typename T, typename VT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(PV_SWEEP_WAVES_PER_EU)))
void sweep_kernel(KArgs<T, VT> a) {
    const int b = blockIdx.x;
    const int k = b & 7;
    const int y0 = int((int64_t)a.Ly * k / 8);
    const int ny = int((int64_t)a.Ly * (k + 1) / 8) - y0;
    const int64_t ntl = (int64_t)a.ntx * ny * a.Lz;
    const int64_t t0 = (int64_t)(b >> 3) * a.tpb;
    const int64_t t1 = min(t0 + a.tpb, ntl);
    sweep_block<P, T, VT>(a, b, y0, ny, t0, t1, b == 0);
}

// One sweep over a batch of independent lattices of the same family in a
// single launch: workgroup b serves instance block_inst[b], whose argument
// record (geometry, buffers, scale and shift) is table[instance]; each
// instance's workgroups are consecutive and cover its tiles in order.
// red_step: the step whose moments the records' folded reduction writes.
template <class P, typename T, typename VT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(PV_SWEEP_WAVES_PER_EU)))
void batch_sweep_kernel(const KArgs<T, VT>* __restrict__ table, const int* __restrict__ block_inst,
                        const int* __restrict__ inst_block0, int red_step) {
    const int b = blockIdx.x;
    const int i = __builtin_amdgcn_readfirstlane(block_inst[b]);
    const int lb = b - __builtin_amdgcn_readfirstlane(inst_block0[i]);
    KArgs<T, VT> a = table[i];
    a.red_step = red_step;
    const int64_t ntl = (int64_t)a.ntx * a.Ly * a.Lz;
    const int64_t t0 = (int64_t)lb * a.tpb;
    const int64_t t1 = min(t0 + a.tpb, ntl);
    sweep_block<P, T, VT>(a, b, 0, a.Ly, t0, t1, lb == 0);
}

// ---------------------------------------------------------------------------
// Staged sweep.  A workgroup owns a column tile of TW consecutive elements of
// the rows (m, w) -- w the outer lattice index (z in 3D, y in 2D), m the
// middle one (y in 3D, none in 2D) -- and walks w.  The rows (m, w-1),
// (m, w), (m, w+1), each with one site of x halo on both sides, live in a
// three-slot LDS ring, so a walk fetches every element of its rows once; the
// rows (m -+ 1, w) of 3D lattices, the tile's z (and acc_in) elements and its
// field values are staged per step.  Every global load is a 16-byte chunk
// per lane.  Loads run two steps ahead: step s issues the rows of step s + 2
// into one of two register sets while it computes from LDS, then hands the
// other set (issued one step earlier) to LDS behind a barrier that waits for
// LDS operations only, so loads and y stores stay in flight across steps.
//
// Walks are items of an XCD part (8 parts: split along m when the lattice has
// at least 8 middle rows, along w otherwise).  Items are numbered walk chunk
// first, then strips of st_Bm middle rows, then x tile, then m; the G
// workgroups of a part take items j, j + G, ... so the workgroups resident on
// one XCD walk a compact block of neighbouring columns side by side and read
// each other's rows (m -+ 1, w) and x halos from the same L2.
// ---------------------------------------------------------------------------
template <typename T, int E, int NT = kBlock>
struct Staged {
    static constexpr int NTH = NT;                           // lanes per workgroup
    static constexpr int ES = int(sizeof(cplx<T>));
    static constexpr int CE = 16 / ES;                       // elements per 16-byte chunk
    static constexpr int TW = NT * E;                        // elements per column tile
    static constexpr int TCH = TW / (CE * NT);               // chunks per lane of a row without halo
    static constexpr int RCH = (TW + 2 * STAGED_MAX_SITE + CE * NT - 1) / (CE * NT);  // with halo
    static_assert(TW % (CE * NT) == 0, "a tile must be whole chunks per lane");
    static_assert(NT % 64 == 0 && NT <= 1024, "whole waves");
};

// Barrier for LDS hand-offs only: waits for this wave's LDS operations, not
// for its global loads and stores, so prefetches and y stores stay in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_s_waitcnt(0xc07f);   // gfx9 encoding: lgkmcnt(0), vmcnt and expcnt unlimited
    __builtin_amdgcn_s_barrier();
}

template <typename T>
__device__ __forceinline__ u32x4 ld_chunk(const void* base, uint32_t boff) {
    return *reinterpret_cast<const u32x4*>(reinterpret_cast<const char*>(base) + boff);
}

template <typename T>
__device__ __forceinline__ u32x4 ld_chunk_nt(const void* base, uint32_t boff) {
    return __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(reinterpret_cast<const char*>(base) + boff));
}

// One step's worth of rows in flight: ring row with halo, z and acc_in
// chunks, field values.  (The side rows of 3D lattices, mostly L2 hits, are
// loaded one step ahead into a single set of their own.)
template <class P, typename T, typename VT, int E, int NT>
struct StagedSet {
    using S = Staged<T, E, NT>;
    u32x4 ring[S::RCH];
    u32x4 z[S::TCH];
    VT v[E];          // stored field entries (converted when handed to LDS)
    int64_t vrow;     // first field entry of the set's row
};

// Side rows hold the tile, or for stencils with hops that have a y and an x
// step (P::SIDE_HALO) the tile with the one-site x halo of ring rows.  They
// are the rows (m -+ 1, w), and for stencils with hops that have a y and a z
// step (P::SIDE_W) also (m -+ 1, w -+ 1): side row idx(dm, dw).
template <class P, typename T, int E, int NT>
struct StagedSide {
    static constexpr int NTR = P::DIM == 3 ? (P::SIDE_W ? 6 : 2) : 0;
    __host__ __device__ static constexpr int idx(int dm, int dw) {
        return (dm < 0 ? 0 : 1) + (P::SIDE_W ? 2 * (dw + 1) : 0);
    }
    static constexpr bool HALO = side_halo<P>();
    static constexpr int SCH = HALO ? Staged<T, E, NT>::RCH : Staged<T, E, NT>::TCH;   // chunks per lane
    static constexpr int SLEN = HALO ? Staged<T, E, NT>::RCH * NT * Staged<T, E, NT>::CE
                                     : Staged<T, E, NT>::TW;                         // LDS elements per row
    u32x4 side[NTR > 0 ? NTR : 1][SCH];
    u32x4 acc[Staged<T, E, NT>::TCH];
};

// ZL: the step reads z (every epilogue but the plain sweep with gamma = 0)
template <class P, typename T, typename VT, int E, bool ACC, int NT, bool ZL = true>
struct StagedCtx {
    using S = Staged<T, E, NT>;
    using Set = StagedSet<P, T, VT, E, NT>;
    using Side = StagedSide<P, T, E, NT>;
    static constexpr int NTR = Side::NTR;
    const KArgs<T, VT>& a;
    cplx<T>* ring;   // [3][seg]
    cplx<T>* tra;    // [NTR][Side::SLEN]
    cplx<T>* zl;     // [TW]
    cplx<T>* al;     // [TW] (ACC only)
    T* vl;           // [E S::NTH]
    int tid, nch, m, wb;
    // per walk: byte offsets inside a row of this lane's ring chunks (x
    // wrapped; open boundaries are applied when computing), row chunks and
    // field entries (clamped into the row)
    uint32_t roff[S::RCH] = {};
    uint32_t soff[S::TCH] = {};
    uint32_t voff[E] = {};
    int vshift = 0;  // element -> field entry: log2 of elements per site or per orbital row

    __device__ __forceinline__ int64_t row_of(int mm, int ww) const {
        return P::DIM == 3 ? (int64_t)ww * a.Ly + mm : (int64_t)ww;
    }
    // Row (mm, ww) after wrapping periodic dimensions; -1 when an open
    // boundary drops it.  Integer selects (no boolean state across blocks),
    // so the row arithmetic stays in scalar registers.
    __device__ __forceinline__ int64_t row_idx(int mm, int ww) const {
        const int Lw = a.st_Lw, Lm = a.st_Lm;
        const int wout = int(ww < 0) | int(ww >= Lw);
        const int mout = int(mm < 0) | int(mm >= Lm);
        const int dead = (wout & (a.st_pw ^ 1)) | (mout & (a.st_pm ^ 1));
        ww += ww < 0 ? Lw : 0;
        ww -= ww >= Lw ? Lw : 0;
        if (ww >= Lw) ww %= Lw;   // w + 3 on a lattice of few planes
        mm += mm < 0 ? Lm : 0;
        mm -= mm >= Lm ? Lm : 0;
        return dead ? int64_t(-1) : row_of(mm, ww);
    }
    __device__ __forceinline__ const cplx<T>* row_ptr(int mm, int ww) const {
        const int64_t r = row_idx(mm, ww);
        return r >= 0 ? a.x + r * a.rowel : a.zero_row;
    }
    __device__ __forceinline__ void setup(int xe0) {
        const int rowel = a.rowel;
        // chunks past the ring row (tile + halo) repeat its last chunk: every
        // lane loads and stores every chunk without branches, and the
        // repeated addresses add no traffic
#pragma unroll
        for (int k = 0; k < S::RCH; ++k) {
            const int q = tid + k * S::NTH;
            int g = xe0 - a.st_site + (q < nch ? q : nch - 1) * S::CE;
            if (g < 0) g += rowel;
            if (g >= rowel) g %= rowel;
            roff[k] = uint32_t(g) * S::ES;
        }
#pragma unroll
        for (int k = 0; k < S::TCH; ++k) {
            const int g = xe0 + (tid + k * S::NTH) * S::CE;
            soff[k] = uint32_t(g < rowel ? g : rowel - S::CE) * S::ES;
        }
        // field entries of the tile: one per site (site field) or per orbital
        // row, clamped into the lattice row
        const int vlen = a.pot_mode == 1 ? a.Lx : a.Lx * P::NO;
#pragma unroll
        for (int k = 0; k < E; ++k) {
            int r = (xe0 >> vshift) + tid + k * S::NTH;
            if (r >= vlen) r = vlen - 1;
            voff[k] = uint32_t(r);
        }
    }
    // Issue the loads of ring row (m, w_ring) and of the per-step rows of
    // outer index w_row (clamped to the walk) into the set.  Every load is
    // unconditional (branch-free code lets the compiler wait for exactly
    // the loads a hand-over needs, keeping the next step's loads in flight).
    __device__ __forceinline__ void issue(Set& st, int w_ring, int w_row) const {
        const cplx<T>* rp = row_ptr(m, w_ring);
#pragma unroll
        for (int k = 0; k < S::RCH; ++k) st.ring[k] = ld_chunk<T>(rp, roff[k]);
        const int wr = w_row < wb ? w_row : wb - 1;
        const int64_t rw = row_of(m, wr);
        const cplx<T>* zr = a.zsrc + rw * a.rowel;
        if constexpr (ZL) {
#pragma unroll
            for (int k = 0; k < S::TCH; ++k) st.z[k] = ld_chunk_nt<T>(zr, soff[k]);
        }
        // stored field entries (a row of the zero row's bytes when the field
        // is absent or generated; those values are not used)
        st.vrow = rw * a.Lx * (a.pot_mode == 1 ? 1 : P::NO);
        const VT* vp = a.field == 1 ? a.V + st.vrow : reinterpret_cast<const VT*>(a.zero_row);
#pragma unroll
        for (int k = 0; k < E; ++k) st.v[k] = vp[voff[k]];
    }
    // Side rows (m -+ 1, w_row) (and (m -+ 1, w_row -+ 1) for SIDE_W),
    // w_row clamped to the walk (3D lattices).
    __device__ __forceinline__ void issue_side(Side& sd, int w_row) const {
        if constexpr (ACC) {
            const int wr = w_row < wb ? w_row : wb - 1;
            const cplx<T>* ar = a.asrc + row_of(m, wr) * a.rowel;
#pragma unroll
            for (int k = 0; k < S::TCH; ++k) sd.acc[k] = ld_chunk_nt<T>(ar, soff[k]);
        }
        if constexpr (NTR > 0) {
            const int wr = w_row < wb ? w_row : wb - 1;
#pragma unroll
            for (int h = 0; h < NTR; ++h) {
                const cplx<T>* sp = row_ptr(m + ((h & 1) ? 1 : -1), wr + (P::SIDE_W ? (h >> 1) - 1 : 0));
                if constexpr (Side::HALO) {
#pragma unroll
                    for (int k = 0; k < Side::SCH; ++k) sd.side[h][k] = ld_chunk<T>(sp, roff[k]);
                } else {
#pragma unroll
                    for (int k = 0; k < Side::SCH; ++k) sd.side[h][k] = ld_chunk<T>(sp, soff[k]);
                }
            }
        }
    }
    __device__ __forceinline__ void commit_side(const Side& sd) const {
        if constexpr (ACC) {
            u32x4* da = reinterpret_cast<u32x4*>(al);
#pragma unroll
            for (int k = 0; k < S::TCH; ++k) da[tid + k * S::NTH] = sd.acc[k];
        }
        if constexpr (NTR > 0) {
#pragma unroll
            for (int h = 0; h < NTR; ++h) {
                u32x4* ds = reinterpret_cast<u32x4*>(tra + h * Side::SLEN);
#pragma unroll
                for (int k = 0; k < Side::SCH; ++k) ds[tid + k * S::NTH] = sd.side[h][k];
            }
        }
    }
    // Hand a set to LDS: ring row into slot, per-step rows into their buffers.
    __device__ __forceinline__ void commit(const Set& st, int slot) const {
        u32x4* d = reinterpret_cast<u32x4*>(ring + slot * a.st_seg);
#pragma unroll
        for (int k = 0; k < S::RCH; ++k) d[tid + k * S::NTH] = st.ring[k];
        if constexpr (ZL) {
            u32x4* dz = reinterpret_cast<u32x4*>(zl);
#pragma unroll
            for (int k = 0; k < S::TCH; ++k) dz[tid + k * S::NTH] = st.z[k];
        }
        if (a.field == 2) {
            // only the entries the tile reads (TW >> vshift: one per site or
            // orbital row) are generated, not one per lane and element
            const int nent = S::TW >> vshift;
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const int q = tid + k * S::NTH;
                if (q < nent) vl[q] = field_at(a, st.vrow + voff[k]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < E; ++k) vl[tid + k * S::NTH] = T(st.v[k]);
        }
    }
    // Ring row (m, ww) alone into a slot (walk prologue).
    __device__ __forceinline__ void ring_now(u32x4 (&r)[S::RCH], int ww, int slot) const {
        const cplx<T>* rp = row_ptr(m, ww);
#pragma unroll
        for (int k = 0; k < S::RCH; ++k) r[k] = ld_chunk<T>(rp, roff[k]);
        u32x4* d = reinterpret_cast<u32x4*>(ring + slot * a.st_seg);
#pragma unroll
        for (int k = 0; k < S::RCH; ++k) d[tid + k * S::NTH] = r[k];
    }
};

// LDS of a staged workgroup: three ring rows with halo (slots padded to
// whole chunks per lane), the side rows of 3D lattices, z (and acc_in) of
// the tile, and the field of its orbital rows (padded to E per lane).
template <typename T, int E, int NT>
__host__ __device__ constexpr int staged_seg() {
    return Staged<T, E, NT>::RCH * NT * Staged<T, E, NT>::CE;
}
template <class P, typename T, int E, int NT>
__host__ __device__ constexpr size_t staged_table_offset(bool acc) {
    return (size_t(3 * staged_seg<T, E, NT>() + StagedSide<P, T, E, NT>::NTR * StagedSide<P, T, E, NT>::SLEN +
                   (1 + (acc ? 1 : 0)) * Staged<T, E, NT>::TW) *
                Staged<T, E, NT>::ES +
            size_t(E * NT) * sizeof(T) + 15) / 16 * 16;
}
// Generic stencils also keep their block entries in LDS: values, then
// offsets, row starts and columns.
template <class P>
struct StagedTable {
    static constexpr int GMAX = (PV_MAX_TERMS_K + 1) * P::NO * P::NO;
    static constexpr int NPTR = (PV_MAX_TERMS_K + 1) * P::NO + 1;
    static constexpr int NINT = 3 * PV_MAX_TERMS_K + NPTR + GMAX;
};
template <class P, typename T, int E, int NT>
__host__ __device__ constexpr size_t staged_lds_bytes_for(bool acc) {
    return staged_table_offset<P, T, E, NT>(acc) +
           (P::FAMILY == FAM_GENERIC
                ? StagedTable<P>::GMAX * sizeof(cplx<T>) + StagedTable<P>::NINT * sizeof(int)
                : 0);
}

template <class P, typename T, typename VT, int E, unsigned EPM, int NT>
__device__ __forceinline__ void staged_block(const KArgs<T, VT>& a, int b_out, int part, int jb, int G) {
    using S = Staged<T, E, NT>;
    constexpr bool ACC = EPM == 0u || (EPM & EP_ACC_ADD) != 0u;
    constexpr bool ZL = (EPM & EP_NO_Z) == 0u;
    using Ctx = StagedCtx<P, T, VT, E, ACC, NT, ZL>;
    using Set = typename Ctx::Set;
    constexpr int NO = P::NO;
    constexpr int NTR = Ctx::NTR;
    constexpr bool GEN = P::FAMILY == FAM_GENERIC;
    extern __shared__ __align__(16) unsigned char smem[];
    const unsigned ep = EPM ? EPM : a.ep;
    const int tid = threadIdx.x;
    const int nb = a.nb;
    const int c = tid & (nb - 1);
    const int o = (tid >> a.lognb) & (NO - 1);
    const int site = a.st_site;
    fused_reduction(a, part == 0 && jb == 0, tid);

    // per-column alpha, beta, gamma only in the run-time epilogue (the
    // specialised ones are launched with uniform values)
    double al = a.alpha, be = a.beta, ga = a.gamma;
    if (EPM == 0u && a.colp != nullptr) {
        al = a.colp[3 * c];
        be = a.colp[3 * c + 1];
        ga = a.colp[3 * c + 2];
    }
    const T alT = T(al), beT = T(be), gaT = T(ga);
    const T er = T(a.eta_re), ei = T(a.eta_im), e0r = T(a.eta0_re), e0i = T(a.eta0_im);
    const int nt_on = GEN ? a.n_terms : P::NT;   // index of the on-site block
    const T dgr = T(a.coef[(((size_t)nt_on * NO + o) * NO + o) * 2]);
    const T dgi = T(a.coef[(((size_t)nt_on * NO + o) * NO + o) * 2 + 1]);
    static constexpr Slots<P> SL{};
    constexpr int NS = SL.n;
    T cre[NS > 0 ? NS : 1], cim[NS > 0 ? NS : 1];
    int dq[NS > 0 ? NS : 1];
    slot_coefficients<P, T, NS>(a.coef, o, nb, cre, cim, dq);
    double dxx = 0.0, dxr = 0.0, dxi = 0.0, dyy = 0.0;

    // generic stencils: offsets and the nonzero entries of every block row
    // (packed by the host after the offsets and the dense blocks) in LDS
    using Tab = StagedTable<P>;
    cplx<T>* g_val = reinterpret_cast<cplx<T>*>(smem + staged_table_offset<P, T, E, NT>(ACC));
    int* g_off = reinterpret_cast<int*>(g_val + Tab::GMAX);
    int* g_ptr = g_off + 3 * PV_MAX_TERMS_K;
    int* g_col = g_ptr + Tab::NPTR;
    if constexpr (GEN) {
        const int nptr = (a.n_terms + 1) * NO + 1;
        const int* gp = a.offs + 3 * a.n_terms;
        const int nnz = gp[nptr - 1];
        const double* gv = a.coef + (size_t)(a.n_terms + 1) * NO * NO * 2;
        for (int i = tid; i < 3 * a.n_terms; i += NT) g_off[i] = a.offs[i];
        for (int i = tid; i < nptr; i += NT) g_ptr[i] = gp[i];
        for (int i = tid; i < nnz; i += NT) {
            g_col[i] = gp[nptr + i];
            g_val[i] = cplx<T>{T(gv[2 * i]), T(gv[2 * i + 1])};
        }
        __syncthreads();
    }

    Ctx cx{a, reinterpret_cast<cplx<T>*>(smem), nullptr, nullptr, nullptr, nullptr, tid, (S::TW + 2 * site) / S::CE, 0, 0};
    cx.vshift = a.pot_mode == 1 ? a.logsite : a.lognb;
    cx.tra = cx.ring + 3 * a.st_seg;
    cx.zl = cx.tra + NTR * Ctx::Side::SLEN;
    cx.al = cx.zl + S::TW;
    cx.vl = reinterpret_cast<T*>(cx.al + (ACC ? S::TW : 0));

    // this part's ranges of m and w
    int m0 = 0, m1 = a.st_Lm, wA = 0, wB = a.st_Lw;
    if (a.st_parts == 8) {
        if (a.st_Lm >= 8) {
            m0 = a.st_Lm * part / 8;
            m1 = a.st_Lm * (part + 1) / 8;
        } else {
            wA = a.st_Lw * part / 8;
            wB = a.st_Lw * (part + 1) / 8;
        }
    }
    const int nm = m1 - m0, nW = wB - wA;
    const int nwc = nW > 0 ? (nW + a.st_C - 1) / a.st_C : 0;
    const int bms = min(a.st_Bm, nm);
    const int per_wc = nm * a.st_nxs;
    const int items = nwc * per_wc;

    for (int j = jb; j < items; j += G) {
        const int wc = j / per_wc;
        const int rem = j - wc * per_wc;
        const int ms = (rem / (bms * a.st_nxs)) * bms;
        const int bm = min(bms, nm - ms);
        const int r2 = rem - ms * a.st_nxs;
        const int xs = r2 / bm;
        cx.m = m0 + ms + (r2 - xs * bm);
        const int xe0 = xs * S::TW;
        cx.setup(xe0);
        const int wa = wA + wc * a.st_C;
        const int wb = min(wa + a.st_C, wB);
        cx.wb = wb;
        const int nsteps = wb - wa;

        // prologue: ring rows wa - 1, wa into slots 0, 1; set A = ring row
        // wa + 1 and the rows of step 0, handed over now; set B = ring row
        // wa + 2 and the rows of step 1, left in flight
        Set A, B;
        typename Ctx::Side SD;
        cx.ring_now(A.ring, wa - 1, 0);
        cx.ring_now(B.ring, wa, 1);
        cx.issue_side(SD, wa);
        cx.issue(A, wa + 1, wa);
        cx.commit(A, 2);
        cx.commit_side(SD);
        cx.issue(B, wa + 2, wa + 1);
        lds_barrier();

        // step s (outer index wa + s): issue the side rows of step s + 1 and
        // `nx` for step s + 2, compute from LDS, hand `cur` (issued for step
        // s + 1) and the side rows over, store.  Issue and hand-over run on
        // every step; past the walk they fetch rows read two steps earlier
        // (cache hits) and fill buffers nobody reads.
        auto step = [&](int s, Set& nx, const Set& cur) {
            const int w = wa + s;
            cx.issue_side(SD, w + 1);
            cx.issue(nx, s + 2 < nsteps ? w + 3 : w + 1, w + 2);
            const cplx<T>* rm = cx.ring + (s % 3) * a.st_seg + site;
            const cplx<T>* r0 = cx.ring + ((s + 1) % 3) * a.st_seg + site;
            const cplx<T>* rp = cx.ring + ((s + 2) % 3) * a.st_seg + site;
            const int64_t rowi = cx.row_of(cx.m, w);
            const int64_t rb = rowi * a.rowel;
            T yr[E], yi[E];
            cplx<T> xs_[E], zv[E], av[E];
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const int l = tid + k * NT;
                const int xe = xe0 + l;
                const int x = xe >> a.logsite;
                const bool xlo = a.px || x > 0, xhi = a.px || x < a.Lx - 1;
                const cplx<T> xc = r0[l];
                const T vs = a.field != 0 ? cx.vl[l >> cx.vshift] : T(0);
                const T d = dgr - beT + vs;
                T hr = d * xc.re - dgi * xc.im;
                T hi = d * xc.im + dgi * xc.re;
                if constexpr (GEN) {
                    // runtime terms: rows (m, w + dw) from the ring with the x
                    // halo, rows (m -+ 1, w) from the side rows (with the x halo
                    // in the instance for hops with a y and an x step; the host
                    // admits no offset with both a y and a z step)
                    for (int tb = 0; tb < a.n_terms; ++tb) {
                        const int dx = g_off[3 * tb], dm = g_off[3 * tb + 1], dw = g_off[3 * tb + 2];
                        // side rows start at the tile (no halo) or one site before it
                        constexpr int side0 = Ctx::Side::HALO ? 1 : 0;
                        const cplx<T>* rw = (dm != 0 ? cx.tra + (dm < 0 ? 0 : Ctx::Side::SLEN) + side0 * site
                                                     : (dw < 0 ? rm : (dw > 0 ? rp : r0))) + l + dx * site;
                        const bool ok = dx < 0 ? xlo : (dx > 0 ? xhi : true);
                        const int e0 = g_ptr[tb * NO + o], e1 = g_ptr[tb * NO + o + 1];
                        for (int e = e0; e < e1; ++e)
                            mac<T>(hr, hi, CC, g_val[e].re, g_val[e].im, zero_unless(ok, rw[(g_col[e] - o) * nb]));
                    }
                    const int e0 = g_ptr[a.n_terms * NO + o], e1 = g_ptr[a.n_terms * NO + o + 1];
                    for (int e = e0; e < e1; ++e)
                        mac<T>(hr, hi, CC, g_val[e].re, g_val[e].im, r0[l + (g_col[e] - o) * nb]);
                } else {
                    sfor<NS>([&](auto jj) {
                        constexpr int jx = decltype(jj)::value;
                        constexpr int t = SL.t[jx];
                        const int dqj = SL.same[jx] ? 0 : dq[jx];   // constant 0 for own-orbital slots
                        cplx<T> v;
                        if constexpr (t == P::NT) {
                            v = r0[l + dqj];
                        } else {
                            constexpr int tt = t < P::NT ? t : 0;
                            constexpr int dx = P::off[tt][0];
                            constexpr int dm = P::DIM == 3 ? P::off[tt][1] : 0;
                            constexpr int dw = P::DIM == 3 ? P::off[tt][2] : P::off[tt][1];
                            if constexpr (dm == 0) {
                                const cplx<T>* rw = dw < 0 ? rm : (dw > 0 ? rp : r0);
                                v = rw[l + dx * site + dqj];
                                if constexpr (dx < 0) v = zero_unless(xlo, v);
                                if constexpr (dx > 0) v = zero_unless(xhi, v);
                            } else {
                                // side rows start at the tile, or one site
                                // before it in the instance with the halo
                                constexpr bool HALO = Ctx::Side::HALO;
                                static_assert(dw == 0 || P::SIDE_W, "side rows at w -+ 1 need SIDE_W");
                                static_assert(dx == 0 || HALO, "x steps on side rows need their halo");
                                constexpr int h = Ctx::Side::idx(dm, dw);
                                v = cx.tra[h * Ctx::Side::SLEN + (HALO ? site : 0) + l + dx * site + dqj];
                                if constexpr (dx < 0) v = zero_unless(xlo, v);
                                if constexpr (dx > 0) v = zero_unless(xhi, v);
                            }
                        }
                        mac<T>(hr, hi, SL.kind[jx], cre[jx], cim[jx], v);
                    });
                }
                xs_[k] = xc;
                yr[k] = hr;
                yi[k] = hi;
                zv[k] = ZL ? cx.zl[l] : cplx<T>{T(0), T(0)};
                av[k] = ACC ? cx.al[l] : cplx<T>{T(0), T(0)};
            }
            lds_barrier();
            cx.commit(cur, (s + 3) % 3);
            cx.commit_side(SD);
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const int xe = xe0 + tid + k * NT;
                if (xe < a.rowel) {
                    const int64_t st = rowi * a.Lx + (xe >> a.logsite);
                    const int64_t gidx = a.ggroup == nb ? st * NO + o : st;
                    epilogue_ep(a, ep, rb + xe, gidx, tid & (a.ggroup - 1), xs_[k], zv[k], av[k], yr[k], yi[k], alT,
                                gaT, er, ei, e0r, e0i, c, dxx, dxr, dxi, dyy);
                }
            }
            lds_barrier();
        };
        int s = 0;
        for (; s + 1 < nsteps; s += 2) {
            step(s, A, B);
            step(s + 1, B, A);
        }
        if (s < nsteps) step(s, A, B);
    }

    if (ep & EP_DOTS) {
        for (int mm = nb; mm < 64; mm <<= 1) {
            dxx += __shfl_xor(dxx, mm);
            dxr += __shfl_xor(dxr, mm);
            dxi += __shfl_xor(dxi, mm);
            dyy += __shfl_xor(dyy, mm);
        }
        __syncthreads();
        double* red = reinterpret_cast<double*>(smem);   // the ring is free after the last barrier
        const int wave = tid >> 6, lane = tid & 63;
        if (lane < nb) {
            red[(wave * PV_MAX_NB_K + lane) * 4 + 0] = dxx;
            red[(wave * PV_MAX_NB_K + lane) * 4 + 1] = dxr;
            red[(wave * PV_MAX_NB_K + lane) * 4 + 2] = dxi;
            red[(wave * PV_MAX_NB_K + lane) * 4 + 3] = dyy;
        }
        __syncthreads();
        if (tid < nb * 4) {
            const int cc = tid >> 2, q = tid & 3;
            double sum = 0.0;
            for (int wv = 0; wv < NT / 64; ++wv) sum += red[(wv * PV_MAX_NB_K + cc) * 4 + q];
            a.partials[((size_t)b_out * nb + cc) * 4 + q] = sum;
        }
    }
}

// Staged sweep over a batch of lattices in one launch: instance i owns the
// workgroups [inst_block0[i], inst_block0[i+1]), a multiple of 8 starting at
// a multiple of 8, split into its 8 XCD parts like a single-lattice launch.
template <class P, typename T, typename VT, int E, unsigned EPM, int NT = kBlock>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(PV_STAGED_WAVES_PER_EU)))
void batch_staged_kernel(const KArgs<T, VT>* __restrict__ table, const int* __restrict__ block_inst,
                         const int* __restrict__ inst_block0, int red_step) {
    const int b = blockIdx.x;
    const int i = __builtin_amdgcn_readfirstlane(block_inst[b]);
    const int b0 = __builtin_amdgcn_readfirstlane(inst_block0[i]);
    const int b1 = __builtin_amdgcn_readfirstlane(inst_block0[i + 1]);
    KArgs<T, VT> a = table[i];
    a.red_step = red_step;
    const int lb = b - b0;
    staged_block<P, T, VT, E, EPM, NT>(a, b, lb & 7, lb >> 3, (b1 - b0) >> 3);
}

// NT lanes per workgroup (256, or 512 for twice the tile length: half the
// relative x halo, one workgroup per CU at the larger shapes)
template <class P, typename T, typename VT, int E, unsigned EPM, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(PV_STAGED_WAVES_PER_EU)))
void staged_kernel(KArgs<T, VT> a) {
    const bool p8 = a.st_parts == 8;
    const int b = blockIdx.x, g = gridDim.x;
    staged_block<P, T, VT, E, EPM, NT>(a, b, p8 ? (b & 7) : 0, p8 ? (b >> 3) : b, p8 ? (g >> 3) : g);
}

#ifndef PV_RTC
// Tiles per workgroup: enough workgroups to keep every CU busy for several
// rounds (>= 32 per CU), at most 64 tiles each (fewer workgroups also means
// fewer partial dot products to reduce).  PV_TILES_PER_BLOCK overrides it
// for tuning runs.
int tiles_per_block(int64_t ntiles) {
    static const int forced = [] {
        const char* e = getenv("PV_TILES_PER_BLOCK");
        return e ? atoi(e) : -1;
    }();
    if (forced > 0) return forced;
    int64_t tpb = ntiles / (256 * 32);
    if (tpb < 1) tpb = 1;
    if (tpb > 64) tpb = 64;
    return int(tpb);
}

template <class P, typename T, typename VT>
int occupancy_blocks() {
    static const int cached = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sweep_kernel<P, T, VT>, kBlock, 0) != hipSuccess || n < 1)
            n = 1;
        return n;
    }();
    return cached;
}

// Kernel arguments from the launch description.  whole_part: one part
// covering the lattice (used by batched launches) instead of 8 XCD parts.
template <class P, typename T, typename VT>
void make_kargs(const SweepParams& p, bool whole_part, KArgs<T, VT>& a) {
    a.x = static_cast<const cplx<T>*>(p.x);
    a.z = static_cast<const cplx<T>*>(p.z);
    a.y = static_cast<cplx<T>*>(p.y);
    a.acc_in = static_cast<const cplx<T>*>(p.acc_in);
    a.acc_out = static_cast<cplx<T>*>(p.acc_out);
    a.zsrc = a.z ? a.z : a.x;
    a.asrc = ((p.ep & EP_ACC_ADD) && a.acc_in) ? a.acc_in : a.x;
    a.V = static_cast<const VT*>(p.V);
    a.field = p.field;
    a.rng_seed = p.rng_seed;
    a.rng_W = p.rng_W;
    a.gw0 = static_cast<const cplx<T>*>(p.gw[0]);
    a.gw1 = static_cast<const cplx<T>*>(p.gw[1]);
    a.gw2 = static_cast<const cplx<T>*>(p.gw[2]);
    a.gcoef = p.gcoef;
    a.grad = p.grad;
    a.gx = p.gx;
    a.gy = p.gy;
    a.ggroup = (p.grad_mode == 2) ? p.nb : P::NO * p.nb;
    a.coef = p.coef;
    a.offs = p.offs;
    a.colp = p.colp;
    a.partials = p.partials;
    a.red_src = p.red_src;
    a.red_out = p.red_out;
    a.red_grid = p.red_grid;
    a.red_mode = p.red_mode;
    a.red_M = p.red_M;
    a.red_step = p.red_step;
    a.red_invD = p.red_invD;
    a.Lx = int(p.L[0]);
    a.Ly = int(p.L[1]);
    a.Lz = int(p.L[2]);
    a.px = p.periodic[0] != 0;
    a.py = p.periodic[1] != 0;
    a.pz = p.periodic[2] != 0;
    a.nb = p.nb;
    int lg = 0;
    while ((1 << lg) < p.nb) ++lg;
    a.lognb = lg;
    int lo = 0;
    while ((1 << lo) < P::NO) ++lo;
    a.logsite = lg + lo;
    a.n_elem = p.L[0] * p.L[1] * p.L[2] * P::NO * p.nb;
    a.rowel = int(p.L[0] * P::NO * p.nb);
    a.ntx = (a.rowel + kBlock - 1) / kBlock;
    a.fd_ntx = make_fastdiv(uint32_t(a.ntx));
    a.BY = p.slab_rows;
    a.fd_slab = make_fastdiv(uint32_t(a.ntx) * uint32_t(a.BY) * uint32_t(p.L[2]));
    a.fd_pf = make_fastdiv(uint32_t(a.ntx) * uint32_t(a.BY));
    a.zero_row = static_cast<const cplx<T>*>(p.zero_row);
    a.ntiles = int64_t(a.ntx) * ((p.L[1] + 7) / 8) * p.L[2];   // tiles of the largest XCD part
    a.n_terms = p.n_terms;
    a.pot_mode = p.pot_mode;
    a.alpha = p.alpha;
    a.beta = p.beta;
    a.gamma = p.gamma;
    a.eta_re = p.eta_re;
    a.eta_im = p.eta_im;
    a.eta0_re = p.eta0_re;
    a.eta0_im = p.eta0_im;
    a.ep = p.ep;
    {
        // a requested count below the default would need more partial-dot
        // rows than a workspace holds: raise it to the default
        const int dflt = tiles_per_block(a.ntiles * 8);
        a.tpb = p.tpb > dflt ? p.tpb : dflt;
    }
    if (whole_part) {
        a.BY = int(p.L[1]);
        a.fd_slab = make_fastdiv(uint32_t(a.ntx) * uint32_t(p.L[1]) * uint32_t(p.L[2]));
        a.fd_pf = make_fastdiv(uint32_t(a.ntx) * uint32_t(p.L[1]));
        a.ntiles = int64_t(a.ntx) * p.L[1] * p.L[2];
        a.tpb = p.tpb > 0 ? p.tpb : tiles_per_block(a.ntiles);
    }
}

int env_int(const char* name, int dflt) {
    const char* e = getenv(name);
    return e ? atoi(e) : dflt;
}

// LDS of a staged kernel instance (independent of nb: tiles are elements)
template <class P, typename T, int E, unsigned EPM, int NT = kBlock>
size_t staged_lds_bytes() {
    return staged_lds_bytes_for<P, T, E, NT>(EPM == 0u || (EPM & EP_ACC_ADD) != 0u);
}

template <class P, typename T, typename VT, int E, int NT = kBlock>
int staged_setup(const SweepParams& p, int G8, bool full_walk, KArgs<T, VT>& a) {
    using S = Staged<T, E, NT>;
    a.st_site = P::NO * p.nb;
    a.st_seg = staged_seg<T, E, NT>();   // ring slot; its first TW + 2 site elements hold the row
    a.st_nxs = (a.rowel + S::TW - 1) / S::TW;
    if (P::DIM == 3) {
        a.st_Lm = a.Ly; a.st_Lw = a.Lz; a.st_pm = a.py; a.st_pw = a.pz;
    } else {
        a.st_Lm = 1; a.st_Lw = a.Ly; a.st_pm = 0; a.st_pw = a.py;
    }
    // the largest part: a split along m when there are 8 middle rows, else along w
    const bool split_m = a.st_Lm >= 8;
    const int nm = split_m ? (a.st_Lm + 7) / 8 : a.st_Lm;
    const int nW = split_m ? a.st_Lw : (a.st_Lw + 7) / 8;
    const int cols = nm * a.st_nxs;
    if (nW < 1) {
        a.st_C = 1;
    } else if (p.st_C > 0) {
        a.st_C = p.st_C < nW ? p.st_C : nW;
    } else if (full_walk) {
        a.st_C = nW;
    } else {
        int nwc = (G8 + cols - 1) / cols;
        if (nwc > nW) nwc = nW;
        a.st_C = (nW + nwc - 1) / nwc;
    }
    const int items = nW < 1 ? 1 : ((nW + a.st_C - 1) / a.st_C) * cols;
    if (G8 > items) G8 = items;
    int bx = int(std::lround(std::sqrt(double(G8) * a.st_site / S::TW)));
    if (bx > a.st_nxs) bx = a.st_nxs;
    if (bx < 1) bx = 1;
    a.st_Bm = p.st_Bm > 0 ? p.st_Bm : (G8 / bx > 1 ? G8 / bx : 1);
    a.st_parts = 8;
    return G8;
}

template <class P, typename T, typename VT, int E, unsigned EPM, int NT = kBlock>
hipError_t launch_staged(SweepParams& p, int num_cus, hipStream_t s) {
    KArgs<T, VT> a;
    make_kargs<P, T, VT>(p, false, a);
    // LDS size and workgroups resident per CU: fixed per kernel instance,
    // set up once (thread-safe initialisation of the local static)
    static const std::pair<hipError_t, int> occ_res = [] {
        const size_t bytes = staged_lds_bytes<P, T, E, EPM, NT>();
        if (bytes > 65536) {
            const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&staged_kernel<P, T, VT, E, EPM, NT>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
            if (e != hipSuccess) return std::make_pair(e, 0);
        }
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, staged_kernel<P, T, VT, E, EPM, NT>, NT, bytes) !=
                hipSuccess || n < 1)
            n = 1;
        return std::make_pair(hipSuccess, n);
    }();
    if (occ_res.first != hipSuccess) return occ_res.first;
    const int occ = occ_res.second;
    const size_t lds = staged_lds_bytes<P, T, E, EPM, NT>();
    int G8 = p.st_G8 > 0 ? p.st_G8 : (num_cus >= 8 ? num_cus / 8 : 1) * occ;
    if (G8 > 256) G8 = 256;
    G8 = staged_setup<P, T, VT, E, NT>(p, G8, false, a);
    p.grid = 8 * G8;
    hipLaunchKernelGGL((staged_kernel<P, T, VT, E, EPM, NT>), dim3(p.grid), dim3(NT), lds, s, a);
    return hipGetLastError();
}

// Epilogue specialisations of the staged kernel: the Chebyshev step with
// fused dots (KPM), the series step (propagation, filters), the plain sweep
// or Chebyshev step without dots (with gamma = 0: no z stream at all), and
// every other combination with the flags read at run time.
template <class P, typename T, typename VT, int E>
hipError_t launch_staged_ep(SweepParams& p, int num_cus, hipStream_t s) {
    constexpr unsigned KPM = EP_STORE_Y | EP_DOTS, SERIES = EP_STORE_Y | EP_ACC_ADD, PLAIN = EP_STORE_Y;
    if (p.colp == nullptr) {
        if constexpr (P::FAMILY != FAM_GENERIC) {
            if (p.st_nt == 512) {
                if (p.ep == KPM) return launch_staged<P, T, VT, E, KPM, 512>(p, num_cus, s);
                if (p.ep == SERIES) return launch_staged<P, T, VT, E, SERIES, 512>(p, num_cus, s);
                if (p.ep == PLAIN)
                    return p.gamma == 0.0 ? launch_staged<P, T, VT, E, PLAIN | EP_NO_Z, 512>(p, num_cus, s)
                                          : launch_staged<P, T, VT, E, PLAIN, 512>(p, num_cus, s);
            }
        }
        if (p.ep == KPM) return launch_staged<P, T, VT, E, KPM>(p, num_cus, s);
        if (p.ep == SERIES) return launch_staged<P, T, VT, E, SERIES>(p, num_cus, s);
        if (p.ep == PLAIN)
            return p.gamma == 0.0 ? launch_staged<P, T, VT, E, PLAIN | EP_NO_Z>(p, num_cus, s)
                                  : launch_staged<P, T, VT, E, PLAIN>(p, num_cus, s);
    }
    if constexpr (sizeof(T) == 8 && E == 2) {
        // the run-time epilogue at two complex128 elements per lane needs more
        // than 256 VGPRs: one element per lane, default walk and workgroups
        SweepParams q = p;
        q.st_C = q.st_Bm = q.st_G8 = 0;
        const hipError_t e = launch_staged<P, T, VT, 1, 0u>(q, num_cus, s);
        p.grid = q.grid;
        return e;
    } else {
        return launch_staged<P, T, VT, E, 0u>(p, num_cus, s);
    }
}

// Epilogues the staged kernel takes by default: plain sweeps, the Chebyshev
// step with dots and the series steps.  The adjoint epilogues (extra vector
// terms and the field gradient) default to the direct kernel, which issues
// their loads together with the neighbour loads.
// Small blocks (below 2^20 elements, cache resident) are launch-latency
// bound, where the direct kernel's single pass beats the staged walks.
bool staged_default(const SweepParams& p) {
    const int64_t elems = p.L[0] * p.L[1] * p.L[2] * p.n_orb * p.nb;
    return (p.ep & (EP_GTERMS | EP_GRAD)) == 0 && elems >= (int64_t(1) << 20);
}

// Elements per lane of a staged launch: one for complex128, two for
// complex64 (one 16-byte chunk per lane and row either way; longer tiles
// need more registers than two resident waves per SIMD allow).
int staged_elems(const SweepParams& p) {
    static const int env_e = env_int("PV_STAGED_E", 0);
    if (p.st_E > 0) return p.st_E;
    if (env_e > 0) return env_e;
    return p.dtype == 0 ? 1 : 2;
}

template <class X>
struct Tag {
    using type = X;
};

// Sweep kernel of a launch: the staged kernel for compiled families, and for
// generic 3D stencils with no offset that has both a y and a z step, when
// the block is 16-byte aligned (its chunk loads); else the direct kernel.
// p.kernel (or PV_SWEEP) 1 forces direct, 2 staged; p.st_E (or PV_STAGED_E)
// selects the elements per lane.
template <class P, typename T, typename VT>
hipError_t launch_typed(SweepParams& p, int num_cus, hipStream_t s) {
    {
        static const int env_kernel = env_int("PV_SWEEP", 0);
        const int kind = p.kernel > 0 ? p.kernel : env_kernel;
        const bool aligned = ((reinterpret_cast<uintptr_t>(p.x) | reinterpret_cast<uintptr_t>(p.zero_row)) & 15) == 0;
        // generic stencils default to staged only on 3D lattices (walks along z)
        const bool can = P::FAMILY != FAM_GENERIC || p.generic_stageable;
        const bool dflt = staged_default(p) && (P::FAMILY != FAM_GENERIC || p.L[2] > 1);
        // a site must be whole 16-byte chunks: ring rows start one site
        // before the tile and wrap by whole chunks (complex64 with
        // n_orb * nb = 1 is half a chunk per site: direct kernel)
        const bool whole = (P::NO * p.nb * int(sizeof(cplx<T>))) % 16 == 0;
        if (can && aligned && whole && P::NO * p.nb <= STAGED_MAX_SITE && (kind == 2 || (kind == 0 && dflt))) {
            const int e = staged_elems(p);
            auto staged = [&](auto pt) -> hipError_t {
                using Q = typename decltype(pt)::type;
                if constexpr (sizeof(T) == 8)
                    return e == 2 ? launch_staged_ep<Q, T, VT, 2>(p, num_cus, s)
                                  : launch_staged_ep<Q, T, VT, 1>(p, num_cus, s);
                else
                    return e == 4 ? launch_staged_ep<Q, T, VT, 4>(p, num_cus, s)
                                  : launch_staged_ep<Q, T, VT, 2>(p, num_cus, s);
            };
            if constexpr (P::FAMILY == FAM_GENERIC) {
                if (p.generic_side_halo) return staged(Tag<PatGeneric<P::NO, true>>{});
            }
            return staged(Tag<P>{});
        }
    }
    (void)num_cus;
    KArgs<T, VT> a;
    make_kargs<P, T, VT>(p, false, a);
    p.grid = int(8 * ((a.ntiles + a.tpb - 1) / a.tpb));
    hipLaunchKernelGGL((sweep_kernel<P, T, VT>), dim3(p.grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <class P>
hipError_t launch_family(SweepParams& p, int num_cus, hipStream_t s) {
    if (p.dtype == 0) {
        if (p.vtype != 0) return hipErrorInvalidValue;
        return launch_typed<P, double, double>(p, num_cus, s);
    }
    if (p.vtype == 0) return launch_typed<P, float, double>(p, num_cus, s);
    return launch_typed<P, float, float>(p, num_cus, s);
}


// Calls f(Tag<T>, Tag<VT>) for the vector and field types of a launch.
template <class F>
hipError_t dispatch_types(int dtype, int vtype, F&& f) {
    if (dtype == 0) {
        if (vtype != 0) return hipErrorInvalidValue;
        return f(Tag<double>{}, Tag<double>{});
    }
    if (vtype == 0) return f(Tag<float>{}, Tag<double>{});
    return f(Tag<float>{}, Tag<float>{});
}

// Argument record of one instance of a batched sweep and its workgroup count.
template <class P>
hipError_t batch_fill_record_fam(const SweepParams& p, int staged, void* dst, int* nblocks) {
    return dispatch_types(p.dtype, p.vtype, [&](auto tt, auto tv) -> hipError_t {
        using T = typename decltype(tt)::type;
        using VT = typename decltype(tv)::type;
        static_assert(sizeof(KArgs<T, VT>) == sizeof(KArgs<double, double>), "record sizes differ");
        KArgs<T, VT> a;
        if constexpr (P::FAMILY != FAM_GENERIC) {
            if (staged) {
                if (P::NO * p.nb > STAGED_MAX_SITE || (P::NO * p.nb * int(sizeof(cplx<T>))) % 16 != 0)
                    return hipErrorInvalidValue;
                make_kargs<P, T, VT>(p, false, a);
                const int e = staged_elems(p);
                const bool w512 = p.st_nt == 512;
                int G8;
                if constexpr (sizeof(T) == 8)
                    G8 = e == 2 ? (w512 ? staged_setup<P, T, VT, 2, 512>(p, 1 << 30, true, a)
                                        : staged_setup<P, T, VT, 2>(p, 1 << 30, true, a))
                                : (w512 ? staged_setup<P, T, VT, 1, 512>(p, 1 << 30, true, a)
                                        : staged_setup<P, T, VT, 1>(p, 1 << 30, true, a));
                else
                    G8 = e == 4 ? (w512 ? staged_setup<P, T, VT, 4, 512>(p, 1 << 30, true, a)
                                        : staged_setup<P, T, VT, 4>(p, 1 << 30, true, a))
                                : (w512 ? staged_setup<P, T, VT, 2, 512>(p, 1 << 30, true, a)
                                        : staged_setup<P, T, VT, 2>(p, 1 << 30, true, a));
                std::memcpy(dst, &a, sizeof(a));
                *nblocks = 8 * G8;
                return hipSuccess;
            }
        }
        make_kargs<P, T, VT>(p, true, a);
        std::memcpy(dst, &a, sizeof(a));
        *nblocks = int((a.ntiles + a.tpb - 1) / a.tpb);
        return hipSuccess;
    });
}

// One step of a batched sweep: every instance's workgroups in one launch.
template <class P>
hipError_t launch_batch_sweep_fam(const SweepParams& p, int staged, const void* table, const int* block_inst,
                                  const int* inst_block0, int grid, int red_step, hipStream_t s) {
    return dispatch_types(p.dtype, p.vtype, [&](auto tt, auto tv) -> hipError_t {
        using T = typename decltype(tt)::type;
        using VT = typename decltype(tv)::type;
        if constexpr (P::FAMILY != FAM_GENERIC) {
            if (staged) {
                constexpr unsigned KPM = EP_STORE_Y | EP_DOTS;
                auto go = [&](auto ke, auto kn) -> hipError_t {
                    constexpr int E = decltype(ke)::value;
                    constexpr int NT = decltype(kn)::value;
                    const size_t lds = staged_lds_bytes<P, T, E, KPM, NT>();
                    if (lds > 65536) {
                        hipError_t e = hipFuncSetAttribute(
                            reinterpret_cast<const void*>(&batch_staged_kernel<P, T, VT, E, KPM, NT>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
                        if (e != hipSuccess) return e;
                    }
                    hipLaunchKernelGGL((batch_staged_kernel<P, T, VT, E, KPM, NT>), dim3(grid), dim3(NT), lds, s,
                                       static_cast<const KArgs<T, VT>*>(table), block_inst, inst_block0, red_step);
                    return hipGetLastError();
                };
                if (p.ep != KPM) return hipErrorInvalidValue;
                const int e = staged_elems(p);
                using I = std::integral_constant<int, 1>;
                using I2 = std::integral_constant<int, 2>;
                using I4 = std::integral_constant<int, 4>;
                using N256 = std::integral_constant<int, kBlock>;
                using N512 = std::integral_constant<int, 512>;
                if constexpr (sizeof(T) == 8) {
                    if (p.st_nt == 512) return e == 2 ? go(I2{}, N512{}) : go(I{}, N512{});
                    return e == 2 ? go(I2{}, N256{}) : go(I{}, N256{});
                } else {
                    if (p.st_nt == 512) return e == 4 ? go(I4{}, N512{}) : go(I2{}, N512{});
                    return e == 4 ? go(I4{}, N256{}) : go(I2{}, N256{});
                }
            }
        }
        hipLaunchKernelGGL((batch_sweep_kernel<P, T, VT>), dim3(grid), dim3(kBlock), 0, s,
                           static_cast<const KArgs<T, VT>*>(table), block_inst, inst_block0, red_step);
        return hipGetLastError();
    });
}

#endif  // PV_RTC
}  // namespace

#ifndef PV_RTC
// One translation unit per family (pv_fam_*.hip) defines these.
#define PV_FAMILY_ENTRY_POINTS(name)                                                                          \
    hipError_t launch_sweep_##name(SweepParams& p, int num_cus, hipStream_t s);                              \
    hipError_t batch_fill_record_##name(const SweepParams& p, int staged, void* dst, int* nblocks);          \
    hipError_t launch_batch_sweep_##name(const SweepParams& p, int staged, const void* table,                \
                                         const int* block_inst, const int* inst_block0, int grid, int red_step, \
                                         hipStream_t s);
PV_FAMILY_ENTRY_POINTS(ti)
PV_FAMILY_ENTRY_POINTS(graphene2)
PV_FAMILY_ENTRY_POINTS(graphene4)
PV_FAMILY_ENTRY_POINTS(weyl)
PV_FAMILY_ENTRY_POINTS(generic)
#undef PV_FAMILY_ENTRY_POINTS
#endif

}  // namespace pv

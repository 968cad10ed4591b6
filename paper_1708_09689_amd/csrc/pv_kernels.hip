// HIP kernels of the library outside the sweep: fixed-order reductions of
// the fused dot products, tall-skinny Gram / rotation, scaling, copies, Bloch
// and random start blocks; and the dispatch of a sweep to its stencil family's
// translation unit (the sweep kernels themselves are in pv_sweep.hpp).
#include "pv_sweep.hpp"

namespace pv {
namespace {

// ------------------------------------------------------------------ reductions

// One wave per block column: the fixed-order reduction shared with the
// reduction folded into a sweep.
__global__ __launch_bounds__(64) void reduce_dots_kernel(const double* __restrict__ partials, int grid, int nb,
                                                         int mode, double* out, int M, int step, double inv_D) {
    reduce_column_wave(partials, grid, nb, blockIdx.x, mode, out, M, step, inv_D, threadIdx.x);
}

// Per-instance fixed-order reduction of a batched sweep: one wave per
// (instance i, column c) sums the partials of the instance's workgroups
// [inst_block0[i], inst_block0[i+1]) and updates mu[i][c][.] (modes 1, 2 of
// reduce_dots_kernel), in the order of the reduction folded into a sweep.
__global__ __launch_bounds__(64) void batch_reduce_kernel(const double* __restrict__ partials,
                                                          const int* __restrict__ inst_block0, int nb, int mode,
                                                          double* mu, int M, int step,
                                                          const double* __restrict__ invD) {
    const int i = blockIdx.x / nb, c = blockIdx.x % nb;
    const int b0 = inst_block0[i], b1 = inst_block0[i + 1];
    reduce_column_wave(partials + (size_t)b0 * nb * 4, b1 - b0, nb, c, mode, mu + (size_t)i * nb * M, M, step,
                       invD[i], threadIdx.x);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void scale_kernel(int64_t n, const cplx<T>* __restrict__ x,
                                                       double re, double im, cplx<T>* __restrict__ y) {
    const T r = T(re), i = T(im);
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock) {
        const cplx<T> v = x[k];
        y[k] = cplx<T>{r * v.re - i * v.im, r * v.im + i * v.re};
    }
}

// ------------------------------------------------------------------ Gram / rotate

constexpr int kGramRows = 16;

// partial G over a strided set of row chunks; pair p = i*ny + j handled by
// thread p % 256, p = tid + 256*k.
template <typename T>
__global__ __launch_bounds__(kBlock) void gram_kernel(const cplx<T>* __restrict__ X,
                                                      const cplx<T>* __restrict__ Y, int64_t rows,
                                                      int nx, int ny, double* __restrict__ partials) {
    __shared__ cplx<double> sx[kGramRows][PV_MAX_NB_K];
    __shared__ cplx<double> sy[kGramRows][PV_MAX_NB_K];
    const int tid = threadIdx.x;
    const int npairs = nx * ny;
    const int kp = (npairs + kBlock - 1) / kBlock;
    double ar[16], ai[16];
    for (int k = 0; k < 16; ++k) { ar[k] = 0.0; ai[k] = 0.0; }
    const int64_t nchunks = (rows + kGramRows - 1) / kGramRows;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t r0 = ch * kGramRows;
        for (int e = tid; e < kGramRows * nx; e += kBlock) {
            const int rr = e / nx, i = e % nx;
            const int64_t r = r0 + rr;
            cplx<double> v{0.0, 0.0};
            if (r < rows) {
                const cplx<T> u = X[r * nx + i];
                v = cplx<double>{double(u.re), double(u.im)};
            }
            sx[rr][i] = v;
        }
        for (int e = tid; e < kGramRows * ny; e += kBlock) {
            const int rr = e / ny, j = e % ny;
            const int64_t r = r0 + rr;
            cplx<double> v{0.0, 0.0};
            if (r < rows) {
                const cplx<T> u = Y[r * ny + j];
                v = cplx<double>{double(u.re), double(u.im)};
            }
            sy[rr][j] = v;
        }
        __syncthreads();
        for (int k = 0; k < kp; ++k) {
            const int p = tid + kBlock * k;
            if (p < npairs) {
                const int i = p / ny, j = p % ny;
                double sr = ar[k], si = ai[k];
                for (int rr = 0; rr < kGramRows; ++rr) {
                    const cplx<double> u = sx[rr][i], v = sy[rr][j];
                    sr += u.re * v.re + u.im * v.im;
                    si += u.re * v.im - u.im * v.re;
                }
                ar[k] = sr;
                ai[k] = si;
            }
        }
        __syncthreads();
    }
    for (int k = 0; k < kp; ++k) {
        const int p = tid + kBlock * k;
        if (p < npairs) {
            partials[((size_t)blockIdx.x * npairs + p) * 2] = ar[k];
            partials[((size_t)blockIdx.x * npairs + p) * 2 + 1] = ai[k];
        }
    }
}

// Gram of a search space kept as nblk column blocks of bw columns each
// (block i at A + i stride): workgroup (group g, block i) takes the row
// chunks g, g + G, ... and accumulates the tiles A_i^H B_j, j in [j0, j0 +
// nj) (j >= i only when hermitian), loading each chunk of A_i once and each
// chunk of B_j once per i; the nblk workgroups of one group run side by side,
// so a chunk of B_j leaves HBM once.  Tile (i, j) of group g goes to
// partials[((i nblk + j) G + g)][bw bw][2].  KP pairs per lane per tile.
template <typename T, int KP>
__global__ __launch_bounds__(kBlock) void block_gram_kernel(const cplx<T>* __restrict__ A,
                                                            const cplx<T>* __restrict__ B, int64_t stride,
                                                            int64_t rows, int bw, int nblk, int j0, int nj,
                                                            int hermitian, double* __restrict__ partials) {
    constexpr int NJ = 32 / KP;
    __shared__ cplx<double> sa[kGramRows][PV_MAX_NB_K];
    __shared__ cplx<double> sb[kGramRows][PV_MAX_NB_K];
    const int tid = threadIdx.x;
    const int i = blockIdx.x % nblk, g = blockIdx.x / nblk, G = gridDim.x / nblk;
    const int np = bw * bw;
    double ar[NJ][KP], ai[NJ][KP];
#pragma unroll
    for (int t = 0; t < NJ; ++t)
#pragma unroll
        for (int k = 0; k < KP; ++k) ar[t][k] = ai[t][k] = 0.0;
    const cplx<T>* Ai = A + (int64_t)i * stride;
    const int64_t nchunks = (rows + kGramRows - 1) / kGramRows;
    for (int64_t ch = g; ch < nchunks; ch += G) {
        const int64_t r0 = ch * kGramRows;
        __syncthreads();
        for (int e = tid; e < kGramRows * bw; e += kBlock) {
            const int rr = e / bw, c = e % bw;
            const int64_t r = r0 + rr;
            cplx<double> v{0.0, 0.0};
            if (r < rows) {
                const cplx<T> u = Ai[r * bw + c];
                v = cplx<double>{double(u.re), double(u.im)};
            }
            sa[rr][c] = v;
        }
#pragma unroll
        for (int t = 0; t < NJ; ++t) {
            const int j = j0 + t;
            if (t >= nj || (hermitian && j < i)) continue;
            const cplx<T>* Bj = B + (int64_t)j * stride;
            __syncthreads();
            for (int e = tid; e < kGramRows * bw; e += kBlock) {
                const int rr = e / bw, c = e % bw;
                const int64_t r = r0 + rr;
                cplx<double> v{0.0, 0.0};
                if (r < rows) {
                    const cplx<T> u = Bj[r * bw + c];
                    v = cplx<double>{double(u.re), double(u.im)};
                }
                sb[rr][c] = v;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                const int p = tid + kBlock * k;
                if (p < np) {
                    const int r = p / bw, c = p % bw;
                    double sr = ar[t][k], si = ai[t][k];
                    for (int rr = 0; rr < kGramRows; ++rr) {
                        const cplx<double> u = sa[rr][r], v = sb[rr][c];
                        sr += u.re * v.re + u.im * v.im;
                        si += u.re * v.im - u.im * v.re;
                    }
                    ar[t][k] = sr;
                    ai[t][k] = si;
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NJ; ++t) {
        const int j = j0 + t;
        if (t >= nj || (hermitian && j < i)) continue;
        double* out = partials + ((size_t)(i * nblk + j) * G + g) * np * 2;
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int p = tid + kBlock * k;
            if (p < np) {
                out[2 * p] = ar[t][k];
                out[2 * p + 1] = ai[t][k];
            }
        }
    }
}

// G[(i bw + r) ns + (j bw + c)] from the tiles of block_gram_kernel, summed
// over the G groups in a fixed order; with hermitian, tiles below the block
// diagonal are the conjugate transposes of those above it.
__global__ __launch_bounds__(kBlock) void block_gram_reduce_kernel(const double* __restrict__ partials, int G,
                                                                   int bw, int nblk, int hermitian,
                                                                   double* __restrict__ out) {
    const int ns = bw * nblk;
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= ns * ns) return;
    const int row = e / ns, col = e % ns;
    int i = row / bw, r = row % bw, j = col / bw, c = col % bw;
    bool conj = false;
    if (hermitian && j < i) {
        const int ti = i, tr = r;
        i = j; r = c; j = ti; c = tr;
        conj = true;
    }
    const double* t = partials + (size_t)(i * nblk + j) * G * bw * bw * 2;
    const int p = r * bw + c;
    double sr = 0.0, si = 0.0;
    for (int g = 0; g < G; ++g) {
        sr += t[((size_t)g * bw * bw + p) * 2];
        si += t[((size_t)g * bw * bw + p) * 2 + 1];
    }
    out[2 * (size_t)e] = sr;
    out[2 * (size_t)e + 1] = conj ? -si : si;
}

// OUT_j = sum_i IN_i Q[i, j] over column blocks: out block j, row r, column c
// = sum_{i, c'} IN_i[r][c'] Q[(i bw + c') (nout bw) + j bw + c], all output
// blocks in one launch (Q complex FP64, accumulation in FP64).
template <typename T>
__global__ __launch_bounds__(kBlock) void block_rotate_kernel(const cplx<T>* __restrict__ IN, int64_t in_stride,
                                                              const double* __restrict__ Q, int64_t rows, int bw,
                                                              int nin, int nout, cplx<T>* __restrict__ OUT,
                                                              int64_t out_stride) {
    const int64_t per = rows * bw;
    const int64_t n = per * nout;
    const int nso = nout * bw;
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < n; e += (int64_t)gridDim.x * kBlock) {
        const int j = int(e / per);
        const int64_t rem = e - (int64_t)j * per;
        const int64_t r = rem / bw;
        const int c = int(rem - r * bw);
        double sr = 0.0, si = 0.0;
        for (int i = 0; i < nin; ++i) {
            const cplx<T>* x = IN + (int64_t)i * in_stride + r * bw;
            const double* q = Q + ((size_t)(i * bw) * nso + j * bw + c) * 2;
            for (int cc = 0; cc < bw; ++cc) {
                const cplx<T> u = x[cc];
                const double qr = q[(size_t)cc * nso * 2], qi = q[(size_t)cc * nso * 2 + 1];
                sr += double(u.re) * qr - double(u.im) * qi;
                si += double(u.re) * qi + double(u.im) * qr;
            }
        }
        OUT[(int64_t)j * out_stride + rem] = cplx<T>{T(sr), T(si)};
    }
}

// Coefficients of the adjoint source terms of the KPM moments, from their
// cotangent gbar [nb][M] (M = 2N).  With mu_{2k} = 2<w_k,w_k>/D - mu_0 and
// mu_{2k+1} = 2 Re<w_k,w_{k+1}>/D - mu_1, the derivative of L = sum gbar mu
// with respect to w_k is (as a sum of terms coef_j w_{k-1+j}, j = 0, 1, 2)
//   j = 0: 2 gbar_{2k-1}, or for k = 1 ghat_1 = gbar_1 - sum_{n=1}^{N-1} gbar_{2n+1};
//   j = 1: 4 gbar_{2k} (k < N);   j = 2: 2 gbar_{2k+1} (k < N);
// each divided by D.  table[k][j][c] complex (imaginary parts zero), k = 0..N
// (row 0 unused, zero).  One thread per (k, c); ghat_1 summed in order of n.
__global__ __launch_bounds__(kBlock) void kpm_adjoint_table_kernel(const double* __restrict__ gbar, int nb, int M,
                                                                  double invD, double* __restrict__ table) {
    const int N = M / 2;
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= (N + 1) * nb) return;
    const int k = e / nb, c = e % nb;
    const double* gc = gbar + (size_t)c * M;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    if (k >= 1) {
        if (k == 1) {
            double ghat1 = gc[1];
            for (int n = 1; n <= N - 1; ++n) ghat1 -= gc[2 * n + 1];
            t0 = ghat1 * invD;
        } else {
            t0 = 2.0 * gc[2 * k - 1] * invD;
        }
        t1 = (k < N ? 4.0 * gc[2 * k] : 0.0) * invD;
        t2 = (k < N ? 2.0 * gc[2 * k + 1] : 0.0) * invD;
    }
    double* row = table + (size_t)k * 3 * nb * 2;
    row[(0 * nb + c) * 2] = t0;
    row[(0 * nb + c) * 2 + 1] = 0.0;
    row[(1 * nb + c) * 2] = t1;
    row[(1 * nb + c) * 2 + 1] = 0.0;
    row[(2 * nb + c) * 2] = t2;
    row[(2 * nb + c) * 2 + 1] = 0.0;
}

// out[k] = sum_b partials[b][k], fixed order over b.
__global__ __launch_bounds__(kBlock) void sum_partials_kernel(const double* __restrict__ partials,
                                                              int grid, int n, double* __restrict__ out) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    double s = 0.0;
    for (int b = 0; b < grid; ++b) s += partials[(size_t)b * n + k];
    out[k] = s;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void rotate_kernel(const cplx<T>* __restrict__ X,
                                                        const double* __restrict__ Q, int64_t rows,
                                                        int nx, int ny, int accumulate,
                                                        cplx<T>* __restrict__ Y) {
    const int64_t n = rows * ny;
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < n; e += (int64_t)gridDim.x * kBlock) {
        const int64_t r = e / ny;
        const int j = int(e - r * ny);
        double sr = 0.0, si = 0.0;
        if (accumulate) {
            const cplx<T> y0 = Y[e];
            sr = double(y0.re);
            si = double(y0.im);
        }
        for (int i = 0; i < nx; ++i) {
            const cplx<T> u = X[r * nx + i];
            const double qr = Q[(i * ny + j) * 2], qi = Q[(i * ny + j) * 2 + 1];
            sr += double(u.re) * qr - double(u.im) * qi;
            si += double(u.re) * qi + double(u.im) * qr;
        }
        Y[e] = cplx<T>{T(sr), T(si)};
    }
}

// dst[0..n) = 0 for 32-bit words (gradients, zero vectors of the adjoint).
__global__ __launch_bounds__(kBlock) void zero_kernel(uint32_t* __restrict__ dst, int64_t n) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock)
        dst[k] = 0u;
}

// Streaming copy: each lane moves 4 x 16 B per iteration with all loads
// issued before the stores; nontemporal on both sides.
__global__ __launch_bounds__(kBlock) void copy_kernel(const u32x4* __restrict__ src,
                                                      u32x4* __restrict__ dst, int64_t n) {
    const int64_t chunk = 4 * (int64_t)kBlock;
    for (int64_t base = blockIdx.x * chunk; base < n; base += (int64_t)gridDim.x * chunk) {
        u32x4 r[4];
        for (int k = 0; k < 4; ++k) {
            const int64_t i = base + k * kBlock + threadIdx.x;
            if (i < n) r[k] = __builtin_nontemporal_load(src + i);
        }
        for (int k = 0; k < 4; ++k) {
            const int64_t i = base + k * kBlock + threadIdx.x;
            if (i < n) __builtin_nontemporal_store(r[k], dst + i);
        }
    }
}

// Streaming triad over FP64 pairs: y = x + z, the stream mix of one
// Chebyshev step (two reads, one write) without the stencil.
using f64x2 = double __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(kBlock) void triad_kernel(const f64x2* __restrict__ x, const f64x2* __restrict__ z,
                                                       f64x2* __restrict__ y, int64_t n) {
    const int64_t chunk = 4 * (int64_t)kBlock;
    for (int64_t base = blockIdx.x * chunk; base < n; base += (int64_t)gridDim.x * chunk) {
        f64x2 a[4], b[4];
        for (int k = 0; k < 4; ++k) {
            const int64_t i = base + k * kBlock + threadIdx.x;
            if (i < n) {
                a[k] = __builtin_nontemporal_load(x + i);
                b[k] = __builtin_nontemporal_load(z + i);
            }
        }
        for (int k = 0; k < 4; ++k) {
            const int64_t i = base + k * kBlock + threadIdx.x;
            if (i < n) __builtin_nontemporal_store(a[k] + b[k], y + i);
        }
    }
}

// Streaming read: every 16-byte chunk of src is loaded once and folded into
// a per-lane XOR; each wave writes one word (the sink keeps the loads live).
__global__ __launch_bounds__(kBlock) void read_kernel(const u32x4* __restrict__ src, int64_t n,
                                                      uint32_t* __restrict__ sink) {
    const int64_t chunk = 4 * (int64_t)kBlock;
    uint32_t acc = 0;
    for (int64_t base = blockIdx.x * chunk; base < n; base += (int64_t)gridDim.x * chunk) {
        u32x4 r[4];
        for (int k = 0; k < 4; ++k) {
            const int64_t i = base + k * kBlock + threadIdx.x;
            r[k] = i < n ? __builtin_nontemporal_load(src + i) : u32x4{0u, 0u, 0u, 0u};
        }
        for (int k = 0; k < 4; ++k) acc ^= r[k].x ^ r[k].y ^ r[k].z ^ r[k].w;
    }
    for (int d = 32; d > 0; d >>= 1) acc ^= uint32_t(__shfl_xor(int(acc), d));
    if ((threadIdx.x & 63) == 0) sink[blockIdx.x * (kBlock / 64) + threadIdx.x / 64] = acc;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void column_copy_kernel(const cplx<T>* __restrict__ src, int src_ld,
                                                           int src_col, cplx<T>* __restrict__ dst, int dst_ld,
                                                           int dst_col, int ncols, int64_t n, double re, double im) {
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < n; e += (int64_t)gridDim.x * kBlock) {
        const int64_t r = e / ncols;
        const int c = int(e - r * ncols);
        const cplx<T> v = src[r * src_ld + src_col + c];
        dst[r * dst_ld + dst_col + c] = cplx<T>{T(re * v.re - im * v.im), T(re * v.im + im * v.re)};
    }
}

// Bloch start columns (one element per lane).
template <typename T>
__global__ __launch_bounds__(kBlock) void bloch_kernel(cplx<T>* __restrict__ out, int64_t n, int n_orb, int nb,
                                                     int Lx, int Ly, BlochCols cols, int axis, int64_t index) {
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < n; e += (int64_t)gridDim.x * kBlock) {
        const int c = int(e % nb);
        const int64_t r = e / nb;
        const int o = int(r % n_orb);
        const int64_t s = r / n_orb;
        const int64_t x = s % Lx, y = (s / Lx) % Ly, z = s / ((int64_t)Lx * Ly);
        const int64_t coord = axis == 0 ? x : (axis == 1 ? y : z);
        double re = 0.0, im = 0.0;
        if (o == cols.orb[c] && (axis < 0 || coord == index)) {
            const double ph = cols.k[c][0] * double(x) + cols.k[c][1] * double(y) + cols.k[c][2] * double(z);
            sincos(ph, &im, &re);
        }
        out[e] = cplx<T>{T(re), T(im)};
    }
}

// Random start blocks (one element per lane): element e takes the
// generator's output for index i0 + e; a random phase exp(2 pi i u) from its
// top 53 bits, or the Z4 phase i^k from its top two.
template <typename T, int KIND>
__global__ __launch_bounds__(kBlock) void random_block_kernel(cplx<T>* __restrict__ out, int64_t n, uint64_t seed,
                                                            uint64_t i0) {
    constexpr double kTwoPi = 6.283185307179586;   // the double nearest 2 pi
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < n; e += (int64_t)gridDim.x * kBlock) {
        const uint64_t z = splitmix64_at(seed, i0 + uint64_t(e));
        double re, im;
        if constexpr (KIND == 0) {
            const double u = double(z >> 11) * 0x1.0p-53;
            sincos(kTwoPi * u, &im, &re);
        } else {
            const int k = int(z >> 62);
            re = k == 0 ? 1.0 : (k == 2 ? -1.0 : 0.0);
            im = k == 1 ? 1.0 : (k == 3 ? -1.0 : 0.0);
        }
        out[e] = cplx<T>{T(re), T(im)};
    }
}

}  // namespace

static int elementwise_grid(int64_t n);

hipError_t launch_column_copy(int dtype, int64_t rows, int ncols, const void* src, int src_ld, int src_col,
                              void* dst, int dst_ld, int dst_col, double re, double im, hipStream_t s) {
    const int64_t n = rows * ncols;
    const int g = elementwise_grid(n);
    if (dtype == 0)
        hipLaunchKernelGGL(column_copy_kernel<double>, dim3(g), dim3(kBlock), 0, s,
                           static_cast<const cplx<double>*>(src), src_ld, src_col, static_cast<cplx<double>*>(dst),
                           dst_ld, dst_col, ncols, n, re, im);
    else
        hipLaunchKernelGGL(column_copy_kernel<float>, dim3(g), dim3(kBlock), 0, s,
                           static_cast<const cplx<float>*>(src), src_ld, src_col, static_cast<cplx<float>*>(dst),
                           dst_ld, dst_col, ncols, n, re, im);
    return hipGetLastError();
}

hipError_t launch_bloch(int dtype, int64_t n_sites, int n_orb, int nb, int Lx, int Ly, const BlochCols& cols,
                        int axis, int64_t index, void* out, hipStream_t s) {
    const int64_t n = n_sites * n_orb * nb;
    const int g = elementwise_grid(n);
    if (dtype == 0)
        hipLaunchKernelGGL(bloch_kernel<double>, dim3(g), dim3(kBlock), 0, s, static_cast<cplx<double>*>(out), n,
                           n_orb, nb, Lx, Ly, cols, axis, index);
    else
        hipLaunchKernelGGL(bloch_kernel<float>, dim3(g), dim3(kBlock), 0, s, static_cast<cplx<float>*>(out), n,
                           n_orb, nb, Lx, Ly, cols, axis, index);
    return hipGetLastError();
}

hipError_t launch_random_block(int dtype, int kind, int64_t n, uint64_t seed, uint64_t i0, void* out, hipStream_t s) {
    const int g = elementwise_grid(n);
    if (dtype == 0) {
        auto* o = static_cast<cplx<double>*>(out);
        if (kind == 0)
            hipLaunchKernelGGL((random_block_kernel<double, 0>), dim3(g), dim3(kBlock), 0, s, o, n, seed, i0);
        else
            hipLaunchKernelGGL((random_block_kernel<double, 1>), dim3(g), dim3(kBlock), 0, s, o, n, seed, i0);
    } else {
        auto* o = static_cast<cplx<float>*>(out);
        if (kind == 0)
            hipLaunchKernelGGL((random_block_kernel<float, 0>), dim3(g), dim3(kBlock), 0, s, o, n, seed, i0);
        else
            hipLaunchKernelGGL((random_block_kernel<float, 1>), dim3(g), dim3(kBlock), 0, s, o, n, seed, i0);
    }
    return hipGetLastError();
}

int64_t sweep_grid_max(const int64_t L[3], int n_orb, int nb) {
    const int64_t rowel = L[0] * n_orb * nb;
    const int64_t ntiles = (rowel + kBlock - 1) / kBlock * ((L[1] + 7) / 8) * L[2];
    const int tpb = tiles_per_block(ntiles * 8);
    const int64_t direct = 8 * ((ntiles + tpb - 1) / tpb);
    return direct > 8 * 256 ? direct : 8 * 256;   // staged: at most 256 workgroups per XCD part
}

hipError_t launch_sweep(SweepParams& p, int num_cus, hipStream_t s) {
    if ((p.ep & (EP_ACC_ADD | EP_ACC_INIT)) && p.acc_kernel > 0) {
        // series steps: their own launch shape (an extra stream changes the best one)
        SweepParams q = p;
        q.kernel = p.acc_kernel;
        q.st_E = p.acc_E;
        q.st_nt = p.acc_nt;
        q.st_C = p.acc_C;
        q.st_Bm = p.acc_Bm;
        q.st_G8 = p.acc_G8;
        q.acc_kernel = 0;
        const hipError_t e = launch_sweep(q, num_cus, s);
        p.grid = q.grid;
        return e;
    }
    switch (p.family) {
        case FAM_TI: return launch_sweep_ti(p, num_cus, s);
        case FAM_GRAPHENE2: return launch_sweep_graphene2(p, num_cus, s);
        case FAM_GRAPHENE4: return launch_sweep_graphene4(p, num_cus, s);
        case FAM_WEYL: return launch_sweep_weyl(p, num_cus, s);
        default:
            if (p.cg_src) {
                const hipError_t e = launch_codegen(p, num_cus, s);
                if (e != hipErrorNotReady || !p.cg_nocompile) return e;
            }
            return launch_sweep_generic(p, num_cus, s);
    }
}

hipError_t launch_reduce_dots(const double* partials, int grid, int nb, int mode, double* out, int M,
                              int step, double inv_D, hipStream_t s) {
    hipLaunchKernelGGL(reduce_dots_kernel, dim3(nb), dim3(64), 0, s, partials, grid, nb, mode, out, M, step,
                       inv_D);
    return hipGetLastError();
}

static int elementwise_grid(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return int(g);
}

hipError_t launch_scale_block(int dtype, int64_t n, const void* x, double re, double im, void* y,
                              hipStream_t s) {
    if (dtype == 0)
        hipLaunchKernelGGL(scale_kernel<double>, dim3(elementwise_grid(n)), dim3(kBlock), 0, s, n,
                           static_cast<const cplx<double>*>(x), re, im, static_cast<cplx<double>*>(y));
    else
        hipLaunchKernelGGL(scale_kernel<float>, dim3(elementwise_grid(n)), dim3(kBlock), 0, s, n,
                           static_cast<const cplx<float>*>(x), re, im, static_cast<cplx<float>*>(y));
    return hipGetLastError();
}

int gram_grid(int64_t rows, int num_cus) {
    int64_t chunks = (rows + kGramRows - 1) / kGramRows;
    int64_t g = (int64_t)num_cus * 2;
    if (g > chunks) g = chunks;
    if (g < 1) g = 1;
    return int(g);
}

hipError_t launch_gram(int dtype, int64_t rows, int nx, int ny, const void* X, const void* Y,
                       double* partials, int grid, double* G, hipStream_t s) {
    if (dtype == 0)
        hipLaunchKernelGGL(gram_kernel<double>, dim3(grid), dim3(kBlock), 0, s,
                           static_cast<const cplx<double>*>(X), static_cast<const cplx<double>*>(Y), rows,
                           nx, ny, partials);
    else
        hipLaunchKernelGGL(gram_kernel<float>, dim3(grid), dim3(kBlock), 0, s,
                           static_cast<const cplx<float>*>(X), static_cast<const cplx<float>*>(Y), rows,
                           nx, ny, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int n = nx * ny * 2;
    hipLaunchKernelGGL(sum_partials_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, partials,
                       grid, n, G);
    return hipGetLastError();
}

int block_gram_groups(int64_t rows, int nblk, int num_cus) {
    const int64_t chunks = (rows + kGramRows - 1) / kGramRows;
    int64_t g = (2 * (int64_t)num_cus + nblk - 1) / nblk;
    if (g > chunks) g = chunks;
    if (g < 1) g = 1;
    return int(g);
}

hipError_t launch_block_gram(int dtype, int64_t rows, int bw, int nblk, const void* A, const void* B,
                             int64_t stride, int hermitian, double* partials, int groups, double* G, hipStream_t s) {
    const int np = bw * bw;
    const int kp = (np + kBlock - 1) / kBlock;   // 1, 4 or 16 for bw <= 64
    const int njmax = 32 / kp;
    for (int j0 = 0; j0 < nblk; j0 += njmax) {
        const int nj = nblk - j0 < njmax ? nblk - j0 : njmax;
        auto go = [&](auto tt, auto kk) {
            using T = typename decltype(tt)::type;
            constexpr int KP = decltype(kk)::value;
            hipLaunchKernelGGL((block_gram_kernel<T, KP>), dim3(groups * nblk), dim3(kBlock), 0, s,
                               static_cast<const cplx<T>*>(A), static_cast<const cplx<T>*>(B), stride, rows, bw,
                               nblk, j0, nj, hermitian, partials);
        };
        auto by_kp = [&](auto tt) {
            if (kp == 1) go(tt, std::integral_constant<int, 1>{});
            else if (kp == 4) go(tt, std::integral_constant<int, 4>{});
            else go(tt, std::integral_constant<int, 16>{});
        };
        if (dtype == 0) by_kp(Tag<double>{});
        else by_kp(Tag<float>{});
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int n = (bw * nblk) * (bw * nblk);
    hipLaunchKernelGGL(block_gram_reduce_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, partials, groups,
                       bw, nblk, hermitian, G);
    return hipGetLastError();
}

hipError_t launch_kpm_adjoint_table(const double* gbar, int nb, int M, double invD, double* table, hipStream_t s) {
    const int n = (M / 2 + 1) * nb;
    hipLaunchKernelGGL(kpm_adjoint_table_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, gbar, nb, M, invD,
                       table);
    return hipGetLastError();
}

hipError_t launch_block_rotate(int dtype, int64_t rows, int bw, int nin, int nout, const void* IN, int64_t in_stride,
                               const double* Q, void* OUT, int64_t out_stride, hipStream_t s) {
    const int g = elementwise_grid(rows * bw * nout);
    if (dtype == 0)
        hipLaunchKernelGGL(block_rotate_kernel<double>, dim3(g), dim3(kBlock), 0, s,
                           static_cast<const cplx<double>*>(IN), in_stride, Q, rows, bw, nin, nout,
                           static_cast<cplx<double>*>(OUT), out_stride);
    else
        hipLaunchKernelGGL(block_rotate_kernel<float>, dim3(g), dim3(kBlock), 0, s,
                           static_cast<const cplx<float>*>(IN), in_stride, Q, rows, bw, nin, nout,
                           static_cast<cplx<float>*>(OUT), out_stride);
    return hipGetLastError();
}

hipError_t launch_rotate(int dtype, int64_t rows, int nx, int ny, const void* X, const double* Q, int accumulate,
                         void* Y, hipStream_t s) {
    const int g = elementwise_grid(rows * ny);
    if (dtype == 0)
        hipLaunchKernelGGL(rotate_kernel<double>, dim3(g), dim3(kBlock), 0, s,
                           static_cast<const cplx<double>*>(X), Q, rows, nx, ny, accumulate,
                           static_cast<cplx<double>*>(Y));
    else
        hipLaunchKernelGGL(rotate_kernel<float>, dim3(g), dim3(kBlock), 0, s,
                           static_cast<const cplx<float>*>(X), Q, rows, nx, ny, accumulate,
                           static_cast<cplx<float>*>(Y));
    return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    const int64_t n = int64_t(bytes / 16);
    int64_t g = (n + 4 * kBlock - 1) / (4 * kBlock);
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(copy_kernel, dim3(int(g)), dim3(kBlock), 0, s, static_cast<const u32x4*>(src),
                       static_cast<u32x4*>(dst), n);
    return hipGetLastError();
}

hipError_t launch_read(const void* src, size_t bytes, void* sink, hipStream_t s) {
    const int64_t n = int64_t(bytes / 16);
    int64_t g = (n + 4 * kBlock - 1) / (4 * kBlock);
    if (g > STREAM_READ_GROUPS) g = STREAM_READ_GROUPS;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(read_kernel, dim3(int(g)), dim3(kBlock), 0, s, static_cast<const u32x4*>(src), n,
                       static_cast<uint32_t*>(sink));
    return hipGetLastError();
}

hipError_t launch_triad(const void* x, const void* z, void* y, size_t bytes, hipStream_t s) {
    const int64_t n = int64_t(bytes / 16);
    int64_t g = (n + 4 * kBlock - 1) / (4 * kBlock);
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(triad_kernel, dim3(int(g)), dim3(kBlock), 0, s, static_cast<const f64x2*>(x),
                       static_cast<const f64x2*>(z), static_cast<f64x2*>(y), n);
    return hipGetLastError();
}

size_t batch_record_bytes() { return sizeof(KArgs<double, double>); }

hipError_t launch_zero(void* dst, size_t bytes, hipStream_t s) {
    const int64_t n = int64_t(bytes / 4);
    hipLaunchKernelGGL(zero_kernel, dim3(elementwise_grid(n)), dim3(kBlock), 0, s, static_cast<uint32_t*>(dst), n);
    return hipGetLastError();
}

hipError_t batch_fill_record(const SweepParams& p, int staged, void* dst, int* nblocks) {
    switch (p.family) {
        case FAM_TI: return batch_fill_record_ti(p, staged, dst, nblocks);
        case FAM_GRAPHENE2: return batch_fill_record_graphene2(p, staged, dst, nblocks);
        case FAM_GRAPHENE4: return batch_fill_record_graphene4(p, staged, dst, nblocks);
        case FAM_WEYL: return batch_fill_record_weyl(p, staged, dst, nblocks);
        default:
            return p.cg_src ? codegen_batch_fill_record(p, staged, dst, nblocks)
                            : batch_fill_record_generic(p, staged, dst, nblocks);
    }
}

hipError_t launch_batch_sweep(const SweepParams& p, int staged, const void* table, const int* block_inst,
                              const int* inst_block0, int grid, int red_step, hipStream_t s) {
    const void* t = table;
    const int* bi = block_inst;
    const int* i0 = inst_block0;
    switch (p.family) {
        case FAM_TI: return launch_batch_sweep_ti(p, staged, t, bi, i0, grid, red_step, s);
        case FAM_GRAPHENE2: return launch_batch_sweep_graphene2(p, staged, t, bi, i0, grid, red_step, s);
        case FAM_GRAPHENE4: return launch_batch_sweep_graphene4(p, staged, t, bi, i0, grid, red_step, s);
        case FAM_WEYL: return launch_batch_sweep_weyl(p, staged, t, bi, i0, grid, red_step, s);
        default:
            return p.cg_src ? launch_batch_codegen(p, staged, t, bi, i0, grid, red_step, s)
                            : launch_batch_sweep_generic(p, staged, t, bi, i0, grid, red_step, s);
    }
}

hipError_t launch_batch_reduce(const double* partials, const int* inst_block0, int n_inst, int nb, int mode,
                               double* mu, int M, int step, const double* invD, hipStream_t s) {
    hipLaunchKernelGGL(batch_reduce_kernel, dim3(n_inst * nb), dim3(64), 0, s, partials, inst_block0, nb, mode, mu,
                       M, step, invD);
    return hipGetLastError();
}

}  // namespace pv

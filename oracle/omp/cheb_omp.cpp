// Oracle (test infrastructure): the Chebyshev step of the fused stencil sweep
// and the KPM moments, over an explicit CSR matrix, in C++17 with OpenMP.
//
// This is the plain definition the matrix-free GPU sweep must reproduce,
// written for the host's cores: the explicit matrix H comes from the oracle's
// assembly of the model equations (Sec. 2), and each row of the block is an
// independent sum over its stored entries.  It shares no code with the
// library; only tests and the CPU baseline of the benchmark call it.
//
//   sweep (Sec. 3.2, generated-code listing, scale_h = alpha, shift_h = beta,
//   scale_z = gamma), per column c of an nb-wide block:
//       y[:, c] = alpha (H x[:, c] - beta x[:, c]) + gamma z[:, c]
//   with the partial dot products <x,x>, <x,y>, <y,y> (<a,b> = sum conj(a) b)
//   accumulated in double precision.
//
//   KPM moments (Sec. 2.2 DOS equation, Sec. 4), per column of r, with
//   H~ = (H - b)/a, w_0 = r, w_1 = H~ w_0, w_{k+1} = 2 H~ w_k - w_{k-1}:
//       mu_0 = <w_0,w_0>/D, mu_1 = Re<w_0,w_1>/D,
//       mu_{2k} = 2<w_k,w_k>/D - mu_0, mu_{2k+1} = 2 Re<w_k,w_{k+1}>/D - mu_1.
#include <omp.h>

#include <complex>
#include <cstdint>
#include <vector>

using cd = std::complex<double>;

extern "C" {

int oracle_omp_threads(void) { return omp_get_max_threads(); }
void oracle_omp_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

// x, z, y: [n_rows][nb] complex (interleaved doubles); z may be NULL when
// gamma == 0 (then it is not read); y must not overlap x.  dots: [nb][4]
// (xx, Re xy, Im xy, yy) or NULL.  Returns 0, or 1 on a bad argument.
int oracle_csr_sweep(int64_t n_rows, const int64_t* indptr, const int64_t* indices, const double* values, int nb,
                     const double* x, const double* z, double* y, double alpha, double beta, double gamma,
                     double* dots) {
    if (n_rows < 0 || nb < 1 || !indptr || !indices || !values || !x || !y || (gamma != 0.0 && !z)) return 1;
    const cd* H = reinterpret_cast<const cd*>(values);
    const cd* X = reinterpret_cast<const cd*>(x);
    const cd* Z = reinterpret_cast<const cd*>(z);
    cd* Y = reinterpret_cast<cd*>(y);
    std::vector<double> acc(static_cast<size_t>(nb) * 4, 0.0);
#pragma omp parallel
    {
        std::vector<double> loc(static_cast<size_t>(nb) * 4, 0.0);
        std::vector<cd> hx(nb);
#pragma omp for schedule(static)
        for (int64_t r = 0; r < n_rows; ++r) {
            for (int c = 0; c < nb; ++c) hx[c] = 0.0;
            for (int64_t k = indptr[r]; k < indptr[r + 1]; ++k) {
                const cd h = H[k];
                const cd* xr = X + indices[k] * nb;
                for (int c = 0; c < nb; ++c) hx[c] += h * xr[c];
            }
            for (int c = 0; c < nb; ++c) {
                const cd xv = X[r * nb + c];
                cd v = alpha * (hx[c] - beta * xv);
                if (gamma != 0.0) v += gamma * Z[r * nb + c];
                Y[r * nb + c] = v;
                const cd xy = std::conj(xv) * v;
                loc[4 * c] += std::norm(xv);
                loc[4 * c + 1] += xy.real();
                loc[4 * c + 2] += xy.imag();
                loc[4 * c + 3] += std::norm(v);
            }
        }
#pragma omp critical
        for (size_t i = 0; i < loc.size(); ++i) acc[i] += loc[i];
    }
    if (dots)
        for (size_t i = 0; i < acc.size(); ++i) dots[i] = acc[i];
    return 0;
}

// mu: [nb][M] (M even, >= 2) for the start block r [n_rows][nb].
int oracle_kpm_moments(int64_t n_rows, const int64_t* indptr, const int64_t* indices, const double* values,
                       int nb, int M, double a, double b, const double* r, double* mu) {
    if (M < 2 || M % 2 || !(a > 0.0) || !r || !mu) return 1;
    const size_t n = static_cast<size_t>(n_rows) * nb * 2;
    std::vector<double> w0(r, r + n), w1(n), d(static_cast<size_t>(nb) * 4);
    const double D = double(n_rows);
    // w_1 = H~ w_0, with <w_0,w_0> and <w_0,w_1>
    if (oracle_csr_sweep(n_rows, indptr, indices, values, nb, w0.data(), nullptr, w1.data(), 1.0 / a, b, 0.0,
                         d.data()))
        return 1;
    std::vector<double> mu0(nb), mu1(nb);
    for (int c = 0; c < nb; ++c) {
        mu0[c] = d[4 * c] / D;
        mu1[c] = d[4 * c + 1] / D;
        mu[static_cast<size_t>(c) * M] = mu0[c];
        mu[static_cast<size_t>(c) * M + 1] = mu1[c];
    }
    // step k: w_{k+1} = 2 H~ w_k - w_{k-1} over w_{k-1}; <w_k,w_k>, <w_k,w_{k+1}>
    for (int k = 1; k < M / 2; ++k) {
        std::vector<double> w2(n);
        if (oracle_csr_sweep(n_rows, indptr, indices, values, nb, w1.data(), w0.data(), w2.data(), 2.0 / a, b,
                             -1.0, d.data()))
            return 1;
        for (int c = 0; c < nb; ++c) {
            mu[static_cast<size_t>(c) * M + 2 * k] = 2.0 * d[4 * c] / D - mu0[c];
            mu[static_cast<size_t>(c) * M + 2 * k + 1] = 2.0 * d[4 * c + 1] / D - mu1[c];
        }
        w0.swap(w1);
        w1.swap(w2);
    }
    return 0;
}

}  // extern "C"

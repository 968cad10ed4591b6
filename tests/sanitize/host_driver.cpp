// Host-only parts of the library under AddressSanitizer and
// UndefinedBehaviorSanitizer (built and run by tests/test_host_sanitizers.py):
// the stencil description parser on the test programs and on deterministic
// mutations of them (truncations, byte replacements, spliced lines), and the
// dense FP64 helpers of Rayleigh-Ritz (Cholesky, triangular inverse, Jacobi
// eigensolver) on random and degenerate Hermitian matrices.  Exit status 0
// when every check holds; the sanitizers abort on the first memory or UB
// error.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "pv_dense.hpp"
#include "pvdtm.h"

// The parser reports errors through this hook of the library.
pv_status pv_fail_status(pv_status st, const char*) { return st; }

namespace {

uint64_t lcg(uint64_t& s) {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return s >> 33;
}

int parse(const std::string& text) {
    int dim = 0, n_orb = 0, n_terms = 0, pot = 0, kind = 0;
    std::vector<int> offs(PV_MAX_TERMS * 3);
    std::vector<double> blocks(PV_MAX_TERMS * PV_MAX_ORB * PV_MAX_ORB * 2), onsite(PV_MAX_ORB * PV_MAX_ORB * 2);
    const double cc[3] = {1.0, 2.0, 0.5};
    return pv_dsl_stencil(text.c_str(), cc, 3, &dim, &n_orb, &n_terms, offs.data(), blocks.data(), onsite.data(),
                          &pot, &kind);
}

int fuzz_dsl(const std::string& text, uint64_t seed) {
    if (parse(text) != PV_OK) {
        std::fprintf(stderr, "golden program did not parse\n");
        return 1;
    }
    int parsed = 0;
    for (size_t n = 0; n <= text.size(); n += 7) parsed += parse(text.substr(0, n)) == PV_OK;
    const char alphabet[] = "0123456789 .-+i|#\nnvcrfe()[]";
    uint64_t s = seed;
    for (int t = 0; t < 400; ++t) {
        std::string m = text;
        const int edits = 1 + int(lcg(s) % 4);
        for (int e = 0; e < edits && !m.empty(); ++e) {
            const size_t pos = lcg(s) % m.size();
            const int op = int(lcg(s) % 3);
            if (op == 0) m[pos] = alphabet[lcg(s) % (sizeof(alphabet) - 1)];
            else if (op == 1) m.erase(pos, 1 + lcg(s) % 5);
            else m.insert(pos, m.substr(lcg(s) % m.size(), 1 + lcg(s) % 20));
        }
        parsed += parse(m) == PV_OK;
    }
    // long junk lines and many repeated statements
    parse(std::string(20000, '9') + "\n");
    std::string rep;
    for (int k = 0; k < 200; ++k) rep += "nn 1 0 0\n0|1|f|1.0\n";
    parse(rep);
    std::printf("parsed %d variants\n", parsed);
    return 0;
}

int check_dense(uint64_t seed) {
    using cd = std::complex<double>;
    uint64_t s = seed;
    auto rnd = [&] { return double(lcg(s) % 2000001) / 1e6 - 1.0; };
    for (int n = 1; n <= 48; n += (n < 8 ? 1 : 9)) {
        // Hermitian with a doubly degenerate pair of eigenvalues built in
        std::vector<cd> A((size_t)n * n);
        for (int i = 0; i < n; ++i)
            for (int j = i; j < n; ++j) {
                const cd v = i == j ? cd(rnd(), 0.0) : cd(rnd(), rnd());
                A[(size_t)i * n + j] = v;
                A[(size_t)j * n + i] = std::conj(v);
            }
        if (n >= 4) {
            for (int i = 0; i < n; ++i) A[(size_t)i * n + 1] = A[(size_t)i * n + 0] = 0.0;
            for (int j = 0; j < n; ++j) A[(size_t)1 * n + j] = A[(size_t)0 * n + j] = 0.0;
            A[0] = A[(size_t)n + 1] = 0.25;
        }
        std::vector<cd> H = A;
        std::vector<double> w;
        std::vector<cd> V;
        pvd::heev_jacobi(n, H, w, V);
        double err = 0.0;
        for (int c = 0; c < n; ++c)
            for (int i = 0; i < n; ++i) {
                cd r = -w[c] * V[(size_t)i * n + c];
                for (int k = 0; k < n; ++k) r += A[(size_t)i * n + k] * V[(size_t)k * n + c];
                err = std::max(err, std::abs(r));
            }
        if (err > 1e-10) {
            std::fprintf(stderr, "eigen residual %g at n = %d\n", err, n);
            return 1;
        }
        // Hermitian positive definite: A^H A + I
        std::vector<cd> P((size_t)n * n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                cd v = i == j ? 1.0 : 0.0;
                for (int k = 0; k < n; ++k) v += std::conj(A[(size_t)k * n + i]) * A[(size_t)k * n + j];
                P[(size_t)i * n + j] = v;
            }
        std::vector<cd> R = P, M;
        if (!pvd::cholesky_upper(n, R)) {
            std::fprintf(stderr, "Cholesky failed at n = %d\n", n);
            return 1;
        }
        pvd::invert_upper(n, R, M);
        double e2 = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                cd v = 0.0;
                for (int k = 0; k < n; ++k) v += R[(size_t)i * n + k] * M[(size_t)k * n + j];
                e2 = std::max(e2, std::abs(v - (i == j ? 1.0 : 0.0)));
            }
        if (e2 > 1e-10) {
            std::fprintf(stderr, "triangular inverse error %g at n = %d\n", e2, n);
            return 1;
        }
        std::vector<cd> Z((size_t)n * n, 0.0);   // not positive definite
        if (pvd::cholesky_upper(n, Z)) {
            std::fprintf(stderr, "Cholesky accepted a zero matrix\n");
            return 1;
        }
    }
    std::printf("dense helpers ok\n");
    return 0;
}

}  // namespace

int main(int argc, char** argv) {
    int bad = 0;
    for (int i = 1; i < argc; ++i) {
        std::ifstream f(argv[i]);
        std::stringstream ss;
        ss << f.rdbuf();
        bad |= fuzz_dsl(ss.str(), 1000 + i);
    }
    bad |= check_dense(7);
    return bad;
}

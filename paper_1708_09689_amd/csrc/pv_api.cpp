// C ABI of the library: argument validation, lattice descriptors, model
// stencils, workspace layout and the host drivers of the Chebyshev
// algorithms.  Every check runs before the first device call, so invalid
// arguments never queue work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "pv_kernels.hpp"
#include "pvdtm.h"

static_assert(pv::PV_MAX_TERMS_K == PV_MAX_TERMS, "kernel-side stencil term limit");

namespace {

thread_local std::string g_err;

pv_status fail(pv_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

pv_status hip_fail(hipError_t e, const char* where) {
    // a generated kernel that did not compile or load says why
    const std::string cg = pv::codegen_error();
    pv::codegen_clear_error();
    if (!cg.empty()) return fail(PV_ERR_HIP, "%s: %s: %s", where, hipGetErrorString(e), cg.c_str());
    return fail(PV_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define PV_HIP(call)                                       \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(e_, #call);  \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int num_cus_of_current_device() {
    static std::mutex mu;
    static std::vector<int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
    if (cache[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        cache[dev] = n;
    }
    return cache[dev];
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

// ---------------------------------------------------------------------------
// lattice object
// ---------------------------------------------------------------------------
struct pv_lattice {
    int dim = 3;
    int64_t L[3] = {1, 1, 1};
    int n_orb = 1;
    int periodic[3] = {1, 1, 1};
    int n_terms = 0;
    std::vector<int> offsets;       // descriptor order
    std::vector<double> blocks;     // descriptor order
    std::vector<double> onsite;
    int pot_mode = 0;
    int family = pv::FAM_GENERIC;
    std::vector<double> packed;     // coefficients in kernel order, on-site last
    std::vector<int> packed_offs;   // generic family
    int64_t n_sites = 0, n_rows = 0;
    // device copies (uploaded on first use on a device)
    std::mutex mu;
    int dev = -1;
    double* d_coef = nullptr;
    int* d_offs = nullptr;
    void* d_zero = nullptr;                            // one x-row of zeros (widest block)
    // borrowed field, or the parameters of the on-the-fly field
    const void* V = nullptr;
    int vtype = 0;
    int rng_on = 0;
    uint64_t rng_seed = 0;
    double rng_W = 0.0;
    // launch shapes per (dtype, log2 nb)
    pv_tuning tune[2][7] = {};
    pv_tuning tune_acc[2][7] = {};   // series steps (autotuned); kernel 0 = follow tune
    // generic stencils: the pattern struct of their generated kernels (empty
    // when a lane's row needs more slots than a kernel holds), and whether
    // sweeps take them (pv_lattice_set_codegen)
    std::string cg_src;
    int codegen = 1;
};

namespace {

template <class P>
bool family_matches(const pv_lattice& l, std::vector<int>& order) {
    if (l.n_orb != P::NO || l.n_terms != P::NT) return false;
    if (P::DIM == 2 && l.L[2] != 1) return false;
    const int NO = P::NO;
    order.assign(P::NT, -1);
    for (int t = 0; t < P::NT; ++t) {
        for (int u = 0; u < l.n_terms; ++u)
            if (l.offsets[3 * u] == P::off[t][0] && l.offsets[3 * u + 1] == P::off[t][1] &&
                l.offsets[3 * u + 2] == P::off[t][2])
                order[t] = u;
        if (order[t] < 0) return false;
    }
    auto fits = [](unsigned char k, double re, double im) {
        if (re != 0.0 && !(k == pv::CR || k == pv::CC)) return false;
        if (im != 0.0 && !(k == pv::CI || k == pv::CC)) return false;
        return true;
    };
    for (int t = 0; t <= P::NT; ++t) {
        const double* B = (t < P::NT) ? &l.blocks[(size_t)order[t] * NO * NO * 2] : l.onsite.data();
        for (int o = 0; o < NO; ++o)
            for (int q = 0; q < NO; ++q) {
                if (t == P::NT && o == q) continue;  // on-site diagonal is always general
                if (!fits(P::code[t][o][q], B[(o * NO + q) * 2], B[(o * NO + q) * 2 + 1])) return false;
            }
    }
    return true;
}

template <class P>
bool try_family(pv_lattice& l) {
    std::vector<int> order;
    if (!family_matches<P>(l, order)) return false;
    const int NO = P::NO;
    l.family = P::FAMILY;
    l.packed.assign((size_t)(P::NT + 1) * NO * NO * 2, 0.0);
    for (int t = 0; t < P::NT; ++t)
        std::memcpy(&l.packed[(size_t)t * NO * NO * 2], &l.blocks[(size_t)order[t] * NO * NO * 2],
                    sizeof(double) * NO * NO * 2);
    std::memcpy(&l.packed[(size_t)P::NT * NO * NO * 2], l.onsite.data(), sizeof(double) * NO * NO * 2);
    l.packed_offs.clear();
    return true;
}

// Side rows a generated 3D pattern stages: with the x halo when some offset
// has a y and an x step, at w -+ 1 too when some offset has a y and a z step.
void codegen_side_flags(const pv_lattice& l, bool& halo, bool& sidew) {
    halo = sidew = false;
    if (l.dim != 3) return;
    for (int t = 0; t < l.n_terms; ++t) {
        const int* d = &l.offsets[3 * t];
        halo = halo || (d[1] != 0 && d[0] != 0);
        sidew = sidew || (d[1] != 0 && d[2] != 0);
    }
}

// Pattern struct of a generic stencil for its generated kernels (Sec. 3.2:
// the DSL's code generation), in the form of the built-in families: the
// offsets in descriptor order and, for every block entry, whether it is
// zero, real, imaginary or complex (the values stay in the coefficient
// table).  Empty when a lane's row would need more slots than a kernel holds.
std::string codegen_pattern(const pv_lattice& l) {
    const int NO = l.n_orb, NT = l.n_terms;
    auto code = [&](int t, int o, int q) {
        const double* e = &l.packed[(((size_t)t * NO + o) * NO + q) * 2];
        if (e[0] == 0.0 && e[1] == 0.0) return 0;
        if (e[1] == 0.0) return 1;
        return e[0] == 0.0 ? 2 : 3;
    };
    int slots = 0;
    for (int t = 0; t <= NT; ++t)
        for (int kd = 1; kd <= 3; ++kd) {
            int K = 0;
            for (int o = 0; o < NO; ++o) {
                int c = 0;
                for (int q = 0; q < NO; ++q)
                    if (!(t == NT && q == o) && code(t, o, q) == kd) ++c;
                K = std::max(K, c);
            }
            slots += K;
        }
    if (slots > pv::MAX_SLOTS_K) return std::string();
    static const char* const kCode[4] = {"CZ", "CR", "CI", "CC"};
    std::string s = "struct PatCG {\n";
    s += "    static constexpr int FAMILY = FAM_CODEGEN, NO = " + std::to_string(NO) + ", NT = " + std::to_string(NT) +
         ", DIM = " + std::to_string(l.dim) + ";\n";
    bool halo, sidew;
    codegen_side_flags(l, halo, sidew);
    s += std::string("    static constexpr bool SIDE_HALO = ") + (halo ? "true" : "false") +
         ", SIDE_W = " + (sidew ? "true" : "false") + ";\n";
    s += "    static constexpr int off[" + std::to_string(std::max(NT, 1)) + "][3] = {";
    for (int t = 0; t < std::max(NT, 1); ++t) {
        const int* d = NT ? &l.offsets[3 * t] : nullptr;
        s += (t ? ", {" : "{") + std::to_string(d ? d[0] : 0) + ", " + std::to_string(d ? d[1] : 0) + ", " +
             std::to_string(d ? d[2] : 0) + "}";
    }
    s += "};\n    static constexpr unsigned char code[NT + 1][NO][NO] = {\n";
    for (int t = 0; t <= NT; ++t) {
        s += "        {";
        for (int o = 0; o < NO; ++o) {
            s += o ? ", {" : "{";
            for (int q = 0; q < NO; ++q) s += std::string(q ? ", " : "") + kCode[code(t, o, q)];
            s += "}";
        }
        s += "},\n";
    }
    s += "    };\n};\n";
    return s;
}

void choose_family(pv_lattice& l) {
    if (try_family<pv::PatTI>(l)) return;
    if (try_family<pv::PatGraphene2>(l)) return;
    if (try_family<pv::PatGraphene4>(l)) return;
    if (try_family<pv::PatWeyl>(l)) return;
    const int NO = l.n_orb;
    l.family = pv::FAM_GENERIC;
    l.packed.assign((size_t)(l.n_terms + 1) * NO * NO * 2, 0.0);
    if (l.n_terms)
        std::memcpy(l.packed.data(), l.blocks.data(), sizeof(double) * l.n_terms * NO * NO * 2);
    std::memcpy(&l.packed[(size_t)l.n_terms * NO * NO * 2], l.onsite.data(), sizeof(double) * NO * NO * 2);
    // The generic kernel walks the nonzero entries of each block row:
    // offsets [n_terms][3], then row starts [(n_terms + 1) NO + 1] and the
    // column of every entry; the entry values follow the dense blocks in
    // `packed`.  Term n_terms is the on-site block without its diagonal.
    l.packed_offs = l.offsets;
    std::vector<int> ptr(1, 0), col;
    std::vector<double> val;
    for (int t = 0; t <= l.n_terms; ++t)
        for (int o = 0; o < NO; ++o) {
            for (int q = 0; q < NO; ++q) {
                if (t == l.n_terms && q == o) continue;
                const double* e = &l.packed[(((size_t)t * NO + o) * NO + q) * 2];
                if (e[0] == 0.0 && e[1] == 0.0) continue;
                col.push_back(q);
                val.push_back(e[0]);
                val.push_back(e[1]);
            }
            ptr.push_back(int(col.size()));
        }
    l.packed_offs.insert(l.packed_offs.end(), ptr.begin(), ptr.end());
    l.packed_offs.insert(l.packed_offs.end(), col.begin(), col.end());
    l.packed.insert(l.packed.end(), val.begin(), val.end());
    l.cg_src = codegen_pattern(l);
}

// Device allocation of the lattice tables.  PV_TEST_FAIL_DEVICE_ALLOC (a test
// hook) makes allocation number k of a set-up fail ("all": every one): 1 the
// coefficient table, 2 the generic offsets, 3 the zero row.
bool device_alloc(void** p, size_t bytes, int k) {
    const char* e = std::getenv("PV_TEST_FAIL_DEVICE_ALLOC");
    if (e && (std::strcmp(e, "all") == 0 || std::atoi(e) == k)) {
        *p = nullptr;
        return false;
    }
    return hipMalloc(p, bytes) == hipSuccess;
}

pv_status ensure_device(pv_lattice* l) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(PV_ERR_NO_DEVICE, "no HIP device: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(l->mu);
    if (l->dev == dev && l->d_coef) return PV_OK;
    if (l->d_coef) { (void)hipFree(l->d_coef); l->d_coef = nullptr; }
    if (l->d_offs) { (void)hipFree(l->d_offs); l->d_offs = nullptr; }
    if (l->d_zero) { (void)hipFree(l->d_zero); l->d_zero = nullptr; }
    const size_t cb = l->packed.size() * sizeof(double);
    if (!device_alloc(reinterpret_cast<void**>(&l->d_coef), cb, 1))
        return fail(PV_ERR_OOM, "coefficient upload: out of memory");
    PV_HIP(hipMemcpy(l->d_coef, l->packed.data(), cb, hipMemcpyHostToDevice));
    if (!l->packed_offs.empty()) {
        const size_t ob = l->packed_offs.size() * sizeof(int);
        if (!device_alloc(reinterpret_cast<void**>(&l->d_offs), ob, 2))
            return fail(PV_ERR_OOM, "offset upload: out of memory");
        PV_HIP(hipMemcpy(l->d_offs, l->packed_offs.data(), ob, hipMemcpyHostToDevice));
    }
    {
        const size_t zb = (size_t)l->L[0] * l->n_orb * PV_MAX_NB * 16;
        if (!device_alloc(&l->d_zero, zb, 3)) return fail(PV_ERR_OOM, "zero row: out of memory");
        PV_HIP(hipMemset(l->d_zero, 0, zb));
    }
    l->dev = dev;
    return PV_OK;
}

// Rows per y-slab: an XCD's slab plane (Lx * BY sites of the nb-wide block)
// is kept near PV_SLAB_BYTES (default 2 MiB) so the +-z neighbour rows of a
// plane are still in that XCD's 4 MiB L2 when the next plane is swept.
int slab_rows(const pv_lattice* l, int dtype, int nb) {
    static const long long target = [] {
        const char* e = getenv("PV_SLAB_BYTES");
        return e ? atoll(e) : (2ll << 20);
    }();
    const long long site = (long long)l->n_orb * nb * (dtype == PV_C128 ? 16 : 8);
    const long long ny_max = (l->L[1] + 7) / 8;
    long long by = target / (l->L[0] * site);
    if (by < 1) by = 1;
    if (by > ny_max) by = ny_max;
    return int(by);
}

size_t elem_bytes(int dtype) { return dtype == PV_C128 ? 16 : 8; }

pv_status check_dtype(const pv_lattice* l, int dtype) {
    if (dtype != PV_C128 && dtype != PV_C64) return fail(PV_ERR_INVALID_ARG, "dtype must be PV_C128 or PV_C64");
    if (dtype == PV_C128 && l->V && l->vtype == PV_F32)
        return fail(PV_ERR_UNSUPPORTED, "complex128 vectors need a float64 on-site field");
    return PV_OK;
}

pv_status check_vec(const void* p, int dtype, const char* name) {
    if (!p) return fail(PV_ERR_INVALID_ARG, "%s is NULL", name);
    if (reinterpret_cast<uintptr_t>(p) % elem_bytes(dtype))
        return fail(PV_ERR_INVALID_ARG, "%s is not %zu-byte aligned", name, elem_bytes(dtype));
    return PV_OK;
}

pv_status check_nb(int nb) {
    if (!is_pow2(nb) || nb > PV_MAX_NB)
        return fail(PV_ERR_UNSUPPORTED, "nb = %d: block width must be a power of two <= %d", nb, PV_MAX_NB);
    return PV_OK;
}

// A generic stencil fits the staged kernel (rows along z in an LDS ring,
// the y neighbours in the plane as side rows, both with an x halo) when no
// offset has both a y and a z step.
int generic_stageable(const pv_lattice* l) {
    if (l->family != pv::FAM_GENERIC || l->dim != 3) return 0;
    for (int t = 0; t < l->n_terms; ++t) {
        const int* d = &l->offsets[3 * t];
        if (d[1] != 0 && d[2] != 0) return 0;
    }
    return 1;
}

// The staged kernel then loads the y neighbours' rows with the x halo too
// when some offset has both a y and an x step.
int generic_side_halo(const pv_lattice* l) {
    if (!generic_stageable(l)) return 0;
    for (int t = 0; t < l->n_terms; ++t) {
        const int* d = &l->offsets[3 * t];
        if (d[1] != 0 && d[0] != 0) return 1;
    }
    return 0;
}

// Sweeps of a generic stencil take its generated kernels unless the lattice
// or PV_CODEGEN=0 turns them off, or the pattern has too many slots.
bool uses_codegen(const pv_lattice* l) {
    static const bool env_on = [] {
        const char* e = std::getenv("PV_CODEGEN");
        return !(e && std::strcmp(e, "0") == 0);
    }();
    return l->family == pv::FAM_GENERIC && l->codegen && !l->cg_src.empty() && env_on;
}

pv::SweepParams base_params(const pv_lattice* l, int dtype, int nb) {
    pv::SweepParams p{};
    p.family = l->family;
    p.dtype = dtype;
    p.vtype = l->vtype;
    p.n_orb = l->n_orb;
    p.n_terms = l->n_terms;
    const bool field = l->V != nullptr || l->rng_on;
    p.pot_mode = field ? l->pot_mode : 0;
    p.field = !field ? 0 : (l->rng_on ? 2 : 1);
    p.rng_seed = l->rng_seed;
    p.rng_W = l->rng_W;
    for (int d = 0; d < 3; ++d) {
        p.L[d] = l->L[d];
        p.periodic[d] = l->periodic[d];
    }
    p.nb = nb;
    p.V = l->pot_mode ? l->V : nullptr;
    p.coef = l->d_coef;
    p.offs = l->d_offs;
    p.generic_stageable = generic_stageable(l);
    p.generic_side_halo = generic_side_halo(l);
    if (uses_codegen(l)) {
        bool halo, sidew;
        codegen_side_flags(*l, halo, sidew);
        p.cg_src = l->cg_src.c_str();
        p.cg_dim = l->dim;
        p.cg_halo = halo;
        p.cg_sidew = sidew;
    }
    return p;
}

int num_cus() {
    const int n = num_cus_of_current_device();
    return n > 0 ? n : 256;
}

int64_t grid_for(const pv_lattice* l, int nb) { return pv::sweep_grid_max(l->L, l->n_orb, nb); }

size_t partial_bytes(const pv_lattice* l, int nb) { return align_up((size_t)grid_for(l, nb) * nb * 4 * sizeof(double)); }
size_t vec_bytes(const pv_lattice* l, int dtype, int nb) {
    return align_up((size_t)l->n_rows * nb * elem_bytes(dtype));
}

// Miller backward recurrence for J_0..J_kmax(z), normalised with
// J_0 + 2 sum_{k>=1} J_{2k} = 1 (Abramowitz & Stegun 9.1.27, 9.1.46).
void bessel_j(double z, int kmax, std::vector<double>& out) {
    out.assign(kmax + 1, 0.0);
    if (z == 0.0) { out[0] = 1.0; return; }
    const bool neg = z < 0.0;
    const double az = std::fabs(z);
    int start = kmax + (int)az + 60;
    start += start & 1;
    std::vector<double> j(start + 2, 0.0);
    j[start] = 1e-30;
    for (int k = start; k > 0; --k) {
        j[k - 1] = (2.0 * k / az) * j[k] - j[k + 1];
        if (std::fabs(j[k - 1]) > 1e250)
            for (int q = k - 1; q <= start; ++q) j[q] *= 1e-250;
    }
    double norm = j[0];
    for (int k = 2; k <= start; k += 2) norm += 2.0 * j[k];
    for (int k = 0; k <= kmax; ++k) out[k] = j[k] / norm * ((neg && (k & 1)) ? -1.0 : 1.0);
}


// Slab height and zero row of a sweep (the device state of the lattice must
// be current).
int log2_nb(int nb) {
    int k = 0;
    while ((1 << k) < nb) ++k;
    return k;
}

pv_status fill_traversal(pv_lattice* l, int dtype, int nb, pv::SweepParams& p) {
    const pv_tuning& t = l->tune[dtype == PV_C128 ? 0 : 1][log2_nb(nb)];
    const int ny_max = int((l->L[1] + 7) / 8);
    p.slab_rows = t.slab_rows > 0 ? std::min(t.slab_rows, ny_max) : slab_rows(l, dtype, nb);
    p.tpb = t.tiles_per_group;
    p.kernel = t.kernel;
    p.st_E = t.elems_per_lane;
    p.st_C = t.walk_planes;
    p.st_Bm = t.strip_rows;
    p.st_G8 = t.groups_per_xcd;
    p.st_nt = t.workgroup_size;
    const pv_tuning& ta = l->tune_acc[dtype == PV_C128 ? 0 : 1][log2_nb(nb)];
    p.acc_kernel = ta.kernel;
    p.acc_E = ta.elems_per_lane;
    p.acc_nt = ta.workgroup_size;
    p.acc_C = ta.walk_planes;
    p.acc_Bm = ta.strip_rows;
    p.acc_G8 = ta.groups_per_xcd;
    p.zero_row = l->d_zero;
    return PV_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// error helpers
// ---------------------------------------------------------------------------
// Error reporting for the other translation units of the library.
pv_status pv_fail_status(pv_status st, const char* msg) { return fail(st, "%s", msg); }

extern "C" const char* pv_last_error(void) { return g_err.c_str(); }

extern "C" const char* pv_status_string(pv_status s) {
    switch (s) {
        case PV_OK: return "ok";
        case PV_ERR_INVALID_ARG: return "invalid argument";
        case PV_ERR_UNSUPPORTED: return "unsupported";
        case PV_ERR_NOT_HERMITIAN: return "stencil is not Hermitian";
        case PV_ERR_WORKSPACE: return "workspace too small";
        case PV_ERR_OOM: return "out of memory";
        case PV_ERR_HIP: return "HIP runtime error";
        case PV_ERR_NONFINITE: return "non-finite result";
        case PV_ERR_NO_DEVICE: return "no device";
        case PV_ERR_NOT_CONVERGED: return "not converged";
    }
    return "unknown status";
}

extern "C" int pv_version(void) { return 1; }

#ifndef PV_SOURCE_HASH
#define PV_SOURCE_HASH "unstamped"
#endif
extern "C" const char* pv_source_hash(void) { return PV_SOURCE_HASH; }

// ---------------------------------------------------------------------------
// model stencils (Sec. 2)
// ---------------------------------------------------------------------------
namespace {
using cd = std::complex<double>;
struct Mat4 {
    cd a[4][4];
};
Mat4 kron2(const cd A[2][2], const cd B[2][2]) {
    Mat4 m;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 2; ++l) m.a[2 * i + k][2 * j + l] = A[i][j] * B[k][l];
    return m;
}
void put_block(double* dst, int no, const cd* m) {
    for (int i = 0; i < no * no; ++i) {
        dst[2 * i] = m[i].real();
        dst[2 * i + 1] = m[i].imag();
    }
}
}  // namespace

extern "C" pv_status pv_model_stencil(int model, const double* params, int* dim, int* n_orb, int* n_terms,
                                      int* offsets, double* blocks, double* onsite, int* pot_mode) {
    if (!dim || !n_orb || !n_terms || !offsets || !blocks || !onsite || !pot_mode)
        return fail(PV_ERR_INVALID_ARG, "pv_model_stencil: NULL output");
    const cd I(0.0, 1.0);
    const cd s0[2][2] = {{1, 0}, {0, 1}};
    const cd sx[2][2] = {{0, 1}, {1, 0}};
    const cd sy[2][2] = {{0, -I}, {I, 0}};
    const cd sz[2][2] = {{1, 0}, {0, -1}};
    const int axis_off[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
    std::memset(blocks, 0, sizeof(double) * PV_MAX_TERMS * PV_MAX_ORB * PV_MAX_ORB * 2);
    std::memset(onsite, 0, sizeof(double) * PV_MAX_ORB * PV_MAX_ORB * 2);
    switch (model) {
        case PV_MODEL_TI: {
            const double t = params ? params[0] : 1.0, m = params ? params[1] : 2.0;
            const double d1 = params ? params[2] : 0.0, d2 = params ? params[3] : 0.0;
            // Gamma^1 = tau_z s0, Gamma^{j+1} = tau_x sigma_j, Gamma^5 = tau_y s0
            const Mat4 G1 = kron2(sz, s0), G5 = kron2(sy, s0);
            const Mat4 Gj[3] = {kron2(sx, sx), kron2(sx, sy), kron2(sx, sz)};
            *dim = 3;
            *n_orb = 4;
            *n_terms = 6;
            *pot_mode = PV_POT_SITE;
            for (int j = 0; j < 3; ++j) {
                cd Am[16], AH[16];  // A = -(t/2)(G1 - i G_{j+1}) carries n -> n + e_j
                for (int r = 0; r < 4; ++r)
                    for (int c = 0; c < 4; ++c) Am[r * 4 + c] = -(t / 2.0) * (G1.a[r][c] - I * Gj[j].a[r][c]);
                for (int r = 0; r < 4; ++r)
                    for (int c = 0; c < 4; ++c) AH[r * 4 + c] = std::conj(Am[c * 4 + r]);
                // (H x)[s] += A x[s - e_j] + A^H x[s + e_j]
                for (int k = 0; k < 3; ++k) {
                    offsets[(2 * j) * 3 + k] = axis_off[2 * j][k];
                    offsets[(2 * j + 1) * 3 + k] = axis_off[2 * j + 1][k];
                }
                put_block(blocks + (2 * j) * 32, 4, Am);
                put_block(blocks + (2 * j + 1) * 32, 4, AH);
            }
            cd E0[16];
            for (int r = 0; r < 4; ++r)
                for (int c = 0; c < 4; ++c) {
                    cd g15 = 0.0;  // [G1, G5]/(2i)
                    for (int k = 0; k < 4; ++k) g15 += G1.a[r][k] * G5.a[k][c] - G5.a[r][k] * G1.a[k][c];
                    g15 /= (2.0 * I);
                    E0[r * 4 + c] = m * G1.a[r][c] + d1 * G5.a[r][c] + d2 * g15;
                }
            put_block(onsite, 4, E0);
            return PV_OK;
        }
        case PV_MODEL_GRAPHENE2: {
            const double t = params ? params[0] : 1.0;
            *dim = 2;
            *n_orb = 2;
            *n_terms = 4;
            *pot_mode = PV_POT_SITE;
            // A(s) couples to B(s), B(s - e_i), B(s - e_j) with -t
            const int off[4][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}};
            std::memcpy(offsets, off, sizeof(off));
            for (int u = 0; u < 4; ++u) {
                double* B = blocks + u * 8;
                if ((u & 1) == 0) B[(0 * 2 + 1) * 2] = -t;  // row A, column B of s - e
                else B[(1 * 2 + 0) * 2] = -t;               // row B, column A of s + e
            }
            onsite[(0 * 2 + 1) * 2] = -t;
            onsite[(1 * 2 + 0) * 2] = -t;
            return PV_OK;
        }
        case PV_MODEL_GRAPHENE4: {
            const double t = params ? params[0] : 1.0;
            *dim = 2;
            *n_orb = 4;
            *n_terms = 4;
            *pot_mode = PV_POT_ORBITAL;
            const int off[4][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}};
            std::memcpy(offsets, off, sizeof(off));
            // T_x carries n -> n + e_x: entries (1,0), (2,3); T_y: (0,3)
            double* Bmx = blocks + 0 * 32;
            double* Bpx = blocks + 1 * 32;
            double* Bmy = blocks + 2 * 32;
            double* Bpy = blocks + 3 * 32;
            Bmx[(1 * 4 + 0) * 2] = -t;
            Bmx[(2 * 4 + 3) * 2] = -t;
            Bpx[(0 * 4 + 1) * 2] = -t;
            Bpx[(3 * 4 + 2) * 2] = -t;
            Bmy[(0 * 4 + 3) * 2] = -t;
            Bpy[(3 * 4 + 0) * 2] = -t;
            for (int a = 0; a < 3; ++a) {
                onsite[(a * 4 + a + 1) * 2] = -t;
                onsite[((a + 1) * 4 + a) * 2] = -t;
            }
            return PV_OK;
        }
        case PV_MODEL_WEYL: {
            const double k0 = params ? params[0] : M_PI / 2.0;
            *dim = 3;
            *n_orb = 2;
            *n_terms = 6;
            *pot_mode = PV_POT_SITE;
            cd A[3][4];
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 2; ++c) {
                    A[0][r * 2 + c] = sx[r][c] / 2.0;
                    A[1][r * 2 + c] = (sx[r][c] + I * sy[r][c]) / 2.0;
                    A[2][r * 2 + c] = (sx[r][c] + I * sz[r][c]) / 2.0;
                }
            for (int j = 0; j < 3; ++j) {
                cd AH[4];
                for (int r = 0; r < 2; ++r)
                    for (int c = 0; c < 2; ++c) AH[r * 2 + c] = std::conj(A[j][c * 2 + r]);
                for (int k = 0; k < 3; ++k) {
                    offsets[(2 * j) * 3 + k] = axis_off[2 * j][k];
                    offsets[(2 * j + 1) * 3 + k] = axis_off[2 * j + 1][k];
                }
                put_block(blocks + (2 * j) * 8, 2, A[j]);
                put_block(blocks + (2 * j + 1) * 8, 2, AH);
            }
            cd E0[4];
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 2; ++c) E0[r * 2 + c] = -sx[r][c] * (2.0 + std::cos(k0));
            put_block(onsite, 2, E0);
            return PV_OK;
        }
        default:
            return fail(PV_ERR_INVALID_ARG, "unknown model %d", model);
    }
}

// ---------------------------------------------------------------------------
// lattice
// ---------------------------------------------------------------------------
extern "C" pv_status pv_lattice_create(const pv_lattice_desc* d, pv_lattice** out) {
    if (!d || !out) return fail(PV_ERR_INVALID_ARG, "pv_lattice_create: NULL argument");
    *out = nullptr;
    if (d->dim != 2 && d->dim != 3) return fail(PV_ERR_INVALID_ARG, "dim must be 2 or 3 (got %d)", d->dim);
    for (int k = 0; k < 3; ++k)
        if (d->L[k] < 1) return fail(PV_ERR_INVALID_ARG, "extent L[%d] = %lld must be >= 1", k, (long long)d->L[k]);
    if (d->dim == 2 && d->L[2] != 1) return fail(PV_ERR_INVALID_ARG, "dim 2 requires L[2] == 1");
    if (d->n_orb != 1 && d->n_orb != 2 && d->n_orb != 4)
        return fail(PV_ERR_UNSUPPORTED, "n_orb = %d: supported are 1, 2, 4", d->n_orb);
    if (d->n_terms < 0 || d->n_terms > PV_MAX_TERMS)
        return fail(PV_ERR_INVALID_ARG, "n_terms = %d outside 0..%d", d->n_terms, PV_MAX_TERMS);
    if (d->n_terms > 0 && (!d->offsets || !d->blocks))
        return fail(PV_ERR_INVALID_ARG, "offsets/blocks NULL with n_terms > 0");
    if (!d->onsite) return fail(PV_ERR_INVALID_ARG, "onsite block is NULL");
    if (d->pot_mode < 0 || d->pot_mode > 2) return fail(PV_ERR_INVALID_ARG, "pot_mode %d invalid", d->pot_mode);
    // overflow guard: elements of a PV_MAX_NB block must index in int64
    const double sites = double(d->L[0]) * double(d->L[1]) * double(d->L[2]);
    if (sites * d->n_orb * PV_MAX_NB * 16.0 > 9.0e18) return fail(PV_ERR_INVALID_ARG, "lattice too large");
    if (sites >= 2147483648.0) return fail(PV_ERR_UNSUPPORTED, "more than 2^31 - 1 sites");
    // the sweeps address an x row of a block with 32-bit element and byte
    // offsets: a row of the widest block (PV_MAX_NB complex128 columns) must
    // stay below 2^31 bytes
    if (double(d->L[0]) * d->n_orb * PV_MAX_NB * 16.0 >= 2147483648.0)
        return fail(PV_ERR_UNSUPPORTED, "L[0] * n_orb = %lld: an x row of a %d-column complex128 block exceeds 2^31 bytes",
                    (long long)d->L[0] * d->n_orb, PV_MAX_NB);
    const int no = d->n_orb;
    for (int t = 0; t < d->n_terms; ++t) {
        const int* o = d->offsets + 3 * t;
        if (o[0] < -1 || o[0] > 1 || o[1] < -1 || o[1] > 1 || o[2] < -1 || o[2] > 1)
            return fail(PV_ERR_UNSUPPORTED, "offset %d = (%d,%d,%d) outside {-1,0,1}^3", t, o[0], o[1], o[2]);
        if (o[0] == 0 && o[1] == 0 && o[2] == 0)
            return fail(PV_ERR_INVALID_ARG, "offset %d is zero (use the on-site block)", t);
        if (d->dim == 2 && o[2] != 0) return fail(PV_ERR_INVALID_ARG, "offset %d has a z component on a 2D lattice", t);
        for (int u = 0; u < t; ++u) {
            const int* p = d->offsets + 3 * u;
            if (p[0] == o[0] && p[1] == o[1] && p[2] == o[2])
                return fail(PV_ERR_INVALID_ARG, "offsets %d and %d coincide", u, t);
        }
    }
    const size_t bsz = (size_t)no * no * 2;
    for (size_t i = 0; i < bsz * d->n_terms; ++i)
        if (!std::isfinite(d->blocks[i])) return fail(PV_ERR_INVALID_ARG, "non-finite block coefficient");
    for (size_t i = 0; i < bsz; ++i)
        if (!std::isfinite(d->onsite[i])) return fail(PV_ERR_INVALID_ARG, "non-finite on-site coefficient");
    if (d->flags & PV_CHECK_HERMITIAN) {
        double scale = 0.0;
        for (size_t i = 0; i < bsz * d->n_terms; ++i) scale = std::max(scale, std::fabs(d->blocks[i]));
        for (size_t i = 0; i < bsz; ++i) scale = std::max(scale, std::fabs(d->onsite[i]));
        const double tol = 1e-14 * std::max(scale, 1.0);
        auto herm_pair = [&](const double* A, const double* B) {  // B == A^H ?
            for (int r = 0; r < no; ++r)
                for (int c = 0; c < no; ++c) {
                    const double* a = A + (r * no + c) * 2;
                    const double* b = B + (c * no + r) * 2;
                    if (std::fabs(a[0] - b[0]) > tol || std::fabs(a[1] + b[1]) > tol) return false;
                }
            return true;
        };
        if (!herm_pair(d->onsite, d->onsite)) return fail(PV_ERR_NOT_HERMITIAN, "on-site block is not Hermitian");
        for (int t = 0; t < d->n_terms; ++t) {
            const int* o = d->offsets + 3 * t;
            int partner = -1;
            for (int u = 0; u < d->n_terms; ++u) {
                const int* p = d->offsets + 3 * u;
                if (p[0] == -o[0] && p[1] == -o[1] && p[2] == -o[2]) partner = u;
            }
            if (partner < 0) return fail(PV_ERR_NOT_HERMITIAN, "offset %d has no opposite offset", t);
            if (!herm_pair(d->blocks + bsz * t, d->blocks + bsz * partner))
                return fail(PV_ERR_NOT_HERMITIAN, "block of offset %d is not the adjoint of its opposite", t);
        }
    }
    pv_lattice* l = new (std::nothrow) pv_lattice();
    if (!l) return fail(PV_ERR_OOM, "host allocation failed");
    l->dim = d->dim;
    for (int k = 0; k < 3; ++k) {
        l->L[k] = d->L[k];
        l->periodic[k] = d->periodic[k] ? 1 : 0;
    }
    l->n_orb = no;
    l->n_terms = d->n_terms;
    l->offsets.assign(d->offsets, d->offsets + 3 * d->n_terms);
    l->blocks.assign(d->blocks, d->blocks + bsz * d->n_terms);
    l->onsite.assign(d->onsite, d->onsite + bsz);
    l->pot_mode = d->pot_mode;
    l->n_sites = d->L[0] * d->L[1] * d->L[2];
    l->n_rows = l->n_sites * no;
    choose_family(*l);
    *out = l;
    return PV_OK;
}

extern "C" void pv_lattice_destroy(pv_lattice* l) {
    if (!l) return;
    if (l->d_coef) (void)hipFree(l->d_coef);
    if (l->d_offs) (void)hipFree(l->d_offs);
    if (l->d_zero) (void)hipFree(l->d_zero);
    delete l;
}

extern "C" pv_status pv_lattice_info(const pv_lattice* l, int64_t* n_sites, int64_t* n_rows, int* family) {
    if (!l) return fail(PV_ERR_INVALID_ARG, "lattice is NULL");
    if (n_sites) *n_sites = l->n_sites;
    if (n_rows) *n_rows = l->n_rows;
    if (family) *family = l->family;
    return PV_OK;
}

extern "C" pv_status pv_lattice_set_potential(pv_lattice* l, const void* V, int rtype) {
    if (!l) return fail(PV_ERR_INVALID_ARG, "lattice is NULL");
    if (rtype != PV_F64 && rtype != PV_F32) return fail(PV_ERR_INVALID_ARG, "rtype must be PV_F64 or PV_F32");
    if (V && l->pot_mode == PV_POT_NONE)
        return fail(PV_ERR_INVALID_ARG, "lattice was created with PV_POT_NONE");
    if (V && reinterpret_cast<uintptr_t>(V) % (rtype == PV_F64 ? 8 : 4))
        return fail(PV_ERR_INVALID_ARG, "potential pointer misaligned");
    l->V = V;
    l->vtype = rtype;
    l->rng_on = 0;
    return PV_OK;
}

extern "C" pv_status pv_lattice_set_random_potential(pv_lattice* l, uint64_t seed, double W) {
    if (!l) return fail(PV_ERR_INVALID_ARG, "lattice is NULL");
    if (l->pot_mode == PV_POT_NONE) return fail(PV_ERR_INVALID_ARG, "lattice was created with PV_POT_NONE");
    if (!std::isfinite(W)) return fail(PV_ERR_INVALID_ARG, "W must be finite");
    l->V = nullptr;
    l->vtype = PV_F64;
    l->rng_on = 1;
    l->rng_seed = seed;
    l->rng_W = W;
    return PV_OK;
}

// ---------------------------------------------------------------------------
// sweep
// ---------------------------------------------------------------------------
extern "C" size_t pv_spmmv_workspace_size(const pv_lattice* l, int dtype, int nb) {
    (void)dtype;
    if (!l || !is_pow2(nb) || nb > PV_MAX_NB) return 0;
    return partial_bytes(l, nb) + align_up(sizeof(double) * 3 * nb);
}

namespace {

// Validation and launch of one fused sweep; the partial dot products go to
// `partials` and non-uniform per-column scales to `colp` (both device
// memory of the caller's choosing, sized by pv_spmmv_workspace_size).
pv_status spmmv_check(pv_lattice* l, int dtype, int nb, const void* x, const void* z, void* y, const double* alpha,
                      const double* beta, const double* gamma, unsigned dot_flags, double* dots, bool& uniform,
                      bool& need_z) {
    if (!l) return fail(PV_ERR_INVALID_ARG, "lattice is NULL");
    pv_status st;
    if ((st = check_dtype(l, dtype)) != PV_OK) return st;
    if ((st = check_nb(nb)) != PV_OK) return st;
    if ((st = check_vec(x, dtype, "x")) != PV_OK) return st;
    if ((st = check_vec(y, dtype, "y")) != PV_OK) return st;
    if (!alpha || !beta || !gamma) return fail(PV_ERR_INVALID_ARG, "alpha/beta/gamma must be host arrays [nb]");
    uniform = true;
    need_z = false;
    for (int c = 0; c < nb; ++c) {
        if (!std::isfinite(alpha[c]) || !std::isfinite(beta[c]) || !std::isfinite(gamma[c]))
            return fail(PV_ERR_INVALID_ARG, "non-finite scale/shift in column %d", c);
        if (alpha[c] != alpha[0] || beta[c] != beta[0] || gamma[c] != gamma[0]) uniform = false;
        if (gamma[c] != 0.0) need_z = true;
    }
    if (need_z && (st = check_vec(z, dtype, "z")) != PV_OK) return st;
    if (x == y || (need_z && x == z)) return fail(PV_ERR_INVALID_ARG, "x must not alias y or z");
    if (dot_flags & ~7u) return fail(PV_ERR_INVALID_ARG, "unknown dot flags 0x%x", dot_flags);
    if (dot_flags && !dots) return fail(PV_ERR_INVALID_ARG, "dots is NULL but dot products were requested");
    return PV_OK;
}

pv_status spmmv_launch(pv_lattice* l, int dtype, int nb, const void* x, const void* z, void* y, const double* alpha,
                       const double* beta, const double* gamma, unsigned dot_flags, double* dots, bool uniform,
                       bool need_z, double* partials, double* colp, hipStream_t s, bool no_compile = false) {
    pv_status st;
    pv::SweepParams p = base_params(l, dtype, nb);
    if ((st = fill_traversal(l, dtype, nb, p)) != PV_OK) return st;
    p.cg_nocompile = no_compile ? 1 : 0;
    p.x = x;
    p.z = need_z ? z : nullptr;
    p.y = y;
    p.alpha = alpha[0];
    p.beta = beta[0];
    p.gamma = gamma[0];
    p.ep = pv::EP_STORE_Y | (dot_flags ? pv::EP_DOTS : 0u);
    p.partials = partials;
    if (!uniform) {
        std::vector<double> h(3 * nb);
        for (int c = 0; c < nb; ++c) {
            h[3 * c] = alpha[c];
            h[3 * c + 1] = beta[c];
            h[3 * c + 2] = gamma[c];
        }
        PV_HIP(hipMemcpyAsync(colp, h.data(), sizeof(double) * 3 * nb, hipMemcpyHostToDevice, s));
        p.colp = colp;
        PV_HIP(pv::launch_sweep(p, num_cus(), s));
        PV_HIP(hipStreamSynchronize(s));  // the host staging buffer h goes out of scope
    } else {
        PV_HIP(pv::launch_sweep(p, num_cus(), s));
    }
    if (dot_flags) PV_HIP(pv::launch_reduce_dots(p.partials, p.grid, nb, 0, dots, 0, 0, 0.0, s));
    return PV_OK;
}

}  // namespace

extern "C" pv_status pv_spmmv(pv_lattice* l, int dtype, int nb, const void* x, const void* z, void* y,
                              const double* alpha, const double* beta, const double* gamma, unsigned dot_flags,
                              double* dots, void* work, size_t work_bytes, void* stream) {
    bool uniform, need_z;
    pv_status st;
    if ((st = spmmv_check(l, dtype, nb, x, z, y, alpha, beta, gamma, dot_flags, dots, uniform, need_z)) != PV_OK)
        return st;
    const size_t need = pv_spmmv_workspace_size(l, dtype, nb);
    if (work_bytes < need || (!work && need)) return fail(PV_ERR_WORKSPACE, "workspace %zu < %zu bytes", work_bytes, need);
    if ((st = ensure_device(l)) != PV_OK) return st;
    char* w = static_cast<char*>(work);
    return spmmv_launch(l, dtype, nb, x, z, y, alpha, beta, gamma, dot_flags, dots, uniform, need_z,
                        reinterpret_cast<double*>(w), reinterpret_cast<double*>(w + partial_bytes(l, nb)),
                        static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------------------
// Allocation-free sweep: the scratch of pv_spmmv (partial dot products,
// per-column scales) in a static device array, one copy per GPU.
// ---------------------------------------------------------------------------
namespace {

static __device__ __align__(256) unsigned char scratch[PV_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch` (looked up once per device,
// with that device current).  The array's name in host code is a host-side
// stand-in and is never passed to a kernel or a copy.
pv_status scratch_of_device(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(PV_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PV_OK;
}

}  // namespace

extern "C" pv_status pv_spmmv_noalloc(pv_lattice* l, int dtype, int nb, const void* x, const void* z, void* y,
                                      const double* alpha, const double* beta, const double* gamma,
                                      unsigned dot_flags, double* dots, void* stream) {
    bool uniform, need_z;
    pv_status st;
    if ((st = spmmv_check(l, dtype, nb, x, z, y, alpha, beta, gamma, dot_flags, dots, uniform, need_z)) != PV_OK)
        return st;
    const size_t need = pv_spmmv_workspace_size(l, dtype, nb);
    if (need > (size_t)PV_NOALLOC_SCRATCH_BYTES)
        return fail(PV_ERR_UNSUPPORTED, "sweep needs %zu bytes of scratch, more than the static %d", need,
                    PV_NOALLOC_SCRATCH_BYTES);
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(PV_ERR_NO_DEVICE, "no HIP device: %s", hipGetErrorString(e));
    {
        // the lattice's device tables are made (allocated) by the first other
        // sweep call on this device; this entry point only uses them
        std::lock_guard<std::mutex> lk(l->mu);
        if (l->dev != dev || !l->d_coef)
            return fail(PV_ERR_INVALID_ARG, "lattice has no device tables on device %d: run one other sweep call "
                                            "(for instance pv_spmmv) on this device first", dev);
    }
    void* ptr = nullptr;
    if ((st = scratch_of_device(dev, &ptr)) != PV_OK) return st;
    char* w = static_cast<char*>(ptr);
    // a generated kernel is taken only when an earlier call loaded it (loading
    // a code object allocates), else the interpreted generic one
    return spmmv_launch(l, dtype, nb, x, z, y, alpha, beta, gamma, dot_flags, dots, uniform, need_z,
                        reinterpret_cast<double*>(w), reinterpret_cast<double*>(w + partial_bytes(l, nb)),
                        static_cast<hipStream_t>(stream), true);
}

// ---------------------------------------------------------------------------
// KPM
// ---------------------------------------------------------------------------
extern "C" size_t pv_kpm_workspace_size(const pv_lattice* l, int dtype, int nb, int M) {
    (void)M;
    if (!l || !is_pow2(nb) || nb > PV_MAX_NB || (dtype != PV_C128 && dtype != PV_C64)) return 0;
    return 2 * partial_bytes(l, nb) + 2 * vec_bytes(l, dtype, nb);
}

namespace {
// Blocks up to this many elements fold each step's moment reduction into the
// next sweep (one launch per step instead of two; their steps are short
// enough for launch latency to matter).
constexpr int64_t kFuseReductionElems = int64_t(1) << 22;
}  // namespace

namespace {

pv_status check_kpm_args(pv_lattice* l, int dtype, int nb, int M, double a, double b, const void* r, const double* mu) {
    if (!l) return fail(PV_ERR_INVALID_ARG, "lattice is NULL");
    pv_status st;
    if ((st = check_dtype(l, dtype)) != PV_OK) return st;
    if ((st = check_nb(nb)) != PV_OK) return st;
    if ((st = check_vec(r, dtype, "r")) != PV_OK) return st;
    if (!mu) return fail(PV_ERR_INVALID_ARG, "mu is NULL");
    if (M < 2 || (M & 1) || M > 65536) return fail(PV_ERR_INVALID_ARG, "M = %d must be even, 2..65536", M);
    if (!(a > 0.0) || !std::isfinite(a) || !std::isfinite(b)) return fail(PV_ERR_INVALID_ARG, "need finite a > 0 and b");
    return PV_OK;
}

// The KPM recurrence with fused dots: w_1 = H~ r, w_{n+1} = 2 H~ w_n - w_{n-1}
// for n < M/2, moments from the per-step dots.  wbuf(k) is the buffer that
// receives w_k (k >= 1); it never aliases w_k's predecessor w_{k-1} (the
// sweep's x), and it may alias w_{k-2} (the sweep's z, updated in place).
template <class WB, class AFTER>
pv_status kpm_forward(pv_lattice* l, int dtype, int nb, int M, double a, double b, const void* r, double* mu,
                      double* part0, double* part1, WB&& wbuf, AFTER&& after, hipStream_t s) {
    pv_status st;
    double* part[2] = {part0, part1};
    pv::SweepParams p = base_params(l, dtype, nb);
    if ((st = fill_traversal(l, dtype, nb, p)) != PV_OK) return st;
    p.ep = pv::EP_STORE_Y | pv::EP_DOTS;
    const double invD = 1.0 / double(l->n_rows);
    const bool fuse = l->n_rows * int64_t(nb) <= kFuseReductionElems;
    // step n's dots go to part[n % 2]; its moments come from the reduction
    // folded into sweep n + 1, or from a reduction launch of their own
    int last_grid = 0;
    auto step_sweep = [&](int n) -> hipError_t {
        p.partials = part[n % 2];
        p.red_src = nullptr;
        if (fuse && n > 0) {
            p.red_src = part[(n - 1) % 2];
            p.red_out = mu;
            p.red_grid = last_grid;
            p.red_mode = n == 1 ? 1 : 2;
            p.red_M = M;
            p.red_step = n - 1;
            p.red_invD = invD;
        }
        hipError_t e = pv::launch_sweep(p, num_cus(), s);
        if (e == hipSuccess && !fuse) e = pv::launch_reduce_dots(p.partials, p.grid, nb, n == 0 ? 1 : 2, mu, M, n, invD, s);
        last_grid = p.grid;
        return e;
    };
    // w_1 = H~ w_0
    p.x = r;
    p.y = wbuf(1);
    p.z = nullptr;
    p.alpha = 1.0 / a;
    p.beta = b;
    p.gamma = 0.0;
    PV_HIP(step_sweep(0));
    PV_HIP(after(1, p.y));
    const void* prev = r;
    const void* cur = p.y;
    p.alpha = 2.0 / a;
    p.gamma = -1.0;
    for (int n = 1; n < M / 2; ++n) {
        void* next = wbuf(n + 1);
        p.x = cur;
        p.z = prev;
        p.y = next;
        PV_HIP(step_sweep(n));
        PV_HIP(after(n + 1, next));
        prev = cur;
        cur = next;
    }
    const int n_last = M / 2 - 1;
    if (fuse)
        PV_HIP(pv::launch_reduce_dots(part[n_last % 2], last_grid, nb, n_last == 0 ? 1 : 2, mu, M, n_last, invD, s));
    return PV_OK;
}

}  // namespace

extern "C" pv_status pv_kpm_moments(pv_lattice* l, int dtype, int nb, int M, double a, double b, const void* r,
                                    double* mu, void* work, size_t work_bytes, void* stream) {
    pv_status st;
    if ((st = check_kpm_args(l, dtype, nb, M, a, b, r, mu)) != PV_OK) return st;
    const size_t need = pv_kpm_workspace_size(l, dtype, nb, M);
    if (!work || work_bytes < need) return fail(PV_ERR_WORKSPACE, "workspace %zu < %zu bytes", work_bytes, need);
    if ((st = ensure_device(l)) != PV_OK) return st;
    char* w = static_cast<char*>(work);
    void* A = w + 2 * partial_bytes(l, nb);
    void* B = static_cast<char*>(A) + vec_bytes(l, dtype, nb);
    // w_k in A for odd k, in B for even k (w_{k+1} overwrites w_{k-1})
    return kpm_forward(l, dtype, nb, M, a, b, r, mu, reinterpret_cast<double*>(w),
                       reinterpret_cast<double*>(w + partial_bytes(l, nb)),
                       [&](int k) { return (k & 1) ? A : B; }, [](int, const void*) { return hipSuccess; },
                       static_cast<hipStream_t>(stream));
}

extern "C" pv_status pv_kpm_dos(int M, const double* mu, double a, double b, int nE, const double* E, double* rho) {
    if (M < 1 || !mu || nE < 0 || (nE && (!E || !rho)) || !(a > 0.0)) return fail(PV_ERR_INVALID_ARG, "pv_kpm_dos: bad arguments");
    for (int n = 0; n < M; ++n)
        if (!std::isfinite(mu[n])) return fail(PV_ERR_NONFINITE, "pv_kpm_dos: moment %d is not finite", n);
    // Jackson damping g_n (Weisse et al. 2006)
    const double q = M_PI / (M + 1);
    std::vector<double> g(M);
    for (int n = 0; n < M; ++n) g[n] = ((M - n + 1) * std::cos(q * n) + std::sin(q * n) / std::tan(q)) / (M + 1);
    for (int e = 0; e < nE; ++e) {
        const double x = (E[e] - b) / a;
        if (!(x > -1.0 && x < 1.0)) { rho[e] = 0.0; continue; }
        // T_n(x) by the three-term recurrence
        double t0 = 1.0, t1 = x, acc = g[0] * mu[0];
        if (M > 1) acc += 2.0 * g[1] * mu[1] * t1;
        for (int n = 2; n < M; ++n) {
            const double t2 = 2.0 * x * t1 - t0;
            acc += 2.0 * g[n] * mu[n] * t2;
            t0 = t1;
            t1 = t2;
        }
        rho[e] = acc / (M_PI * a * std::sqrt(1.0 - x * x));
    }
    return PV_OK;
}

extern "C" pv_status pv_kpm_spectral_function(int nb, int M, const double* mu, double a, double b, double norm,
                                              int nE, const double* E, double* A) {
    if (nb < 1 || M < 1 || !mu || nE < 0 || (nE && (!E || !A)) || !(a > 0.0) || !std::isfinite(norm))
        return fail(PV_ERR_INVALID_ARG, "pv_kpm_spectral_function: bad arguments");
    std::vector<double> rho(nE > 0 ? nE : 1);
    for (int e = 0; e < nE; ++e) A[e] = 0.0;
    for (int c = 0; c < nb; ++c) {
        pv_status st = pv_kpm_dos(M, mu + (size_t)c * M, a, b, nE, E, rho.data());
        if (st != PV_OK) return st;
        for (int e = 0; e < nE; ++e) A[e] += norm * rho[e];
    }
    return PV_OK;
}

extern "C" pv_status pv_bloch_block(pv_lattice* l, int dtype, int nb, const double* k, const int* orbital,
                                    int layer_axis, int64_t layer_index, void* out, void* stream) {
    if (!l) return fail(PV_ERR_INVALID_ARG, "lattice is NULL");
    pv_status st;
    if (dtype != PV_C128 && dtype != PV_C64) return fail(PV_ERR_INVALID_ARG, "dtype must be PV_C128 or PV_C64");
    if ((st = check_nb(nb)) != PV_OK) return st;
    if ((st = check_vec(out, dtype, "out")) != PV_OK) return st;
    if (!k || !orbital) return fail(PV_ERR_INVALID_ARG, "k and orbital are required host arrays [nb]");
    if (layer_axis < -1 || layer_axis > 2) return fail(PV_ERR_INVALID_ARG, "layer_axis must be -1, 0, 1 or 2");
    if (layer_axis >= 0 && (layer_index < 0 || layer_index >= l->L[layer_axis]))
        return fail(PV_ERR_INVALID_ARG, "layer_index %lld outside the lattice", (long long)layer_index);
    pv::BlochCols cols{};
    for (int c = 0; c < nb; ++c) {
        if (orbital[c] < 0 || orbital[c] >= l->n_orb)
            return fail(PV_ERR_INVALID_ARG, "orbital[%d] = %d outside [0, %d)", c, orbital[c], l->n_orb);
        for (int d = 0; d < 3; ++d) {
            if (!std::isfinite(k[3 * c + d])) return fail(PV_ERR_INVALID_ARG, "k[%d] is not finite", c);
            cols.k[c][d] = k[3 * c + d];
        }
        cols.orb[c] = orbital[c];
    }
    int dev;
    if (hipGetDevice(&dev) != hipSuccess) return fail(PV_ERR_NO_DEVICE, "no HIP device");
    PV_HIP(pv::launch_bloch(dtype, l->n_sites, l->n_orb, nb, int(l->L[0]), int(l->L[1]), cols, layer_axis,
                            layer_index, out, static_cast<hipStream_t>(stream)));
    return PV_OK;
}

extern "C" pv_status pv_vector_from_func(pv_lattice* l, int dtype, int nb, pv_vector_func fnc,
                                         pv_vector_func fnc_im, void* parm, uint64_t seed_value, void* out,
                                         void* stream) {
    if (!l) return fail(PV_ERR_INVALID_ARG, "lattice is NULL");
    pv_status st;
    if (dtype != PV_C128 && dtype != PV_C64) return fail(PV_ERR_INVALID_ARG, "dtype must be PV_C128 or PV_C64");
    if ((st = check_nb(nb)) != PV_OK) return st;
    if (!fnc) return fail(PV_ERR_INVALID_ARG, "fnc is NULL");
    if ((st = check_vec(out, dtype, "out")) != PV_OK) return st;
    int dev;
    if (hipGetDevice(&dev) != hipSuccess) return fail(PV_ERR_NO_DEVICE, "no HIP device");
    const size_t n = size_t(l->n_rows) * size_t(nb);
    std::vector<double> h64;
    std::vector<float> h32;
    try {
        if (dtype == PV_C128) h64.resize(2 * n);
        else h32.resize(2 * n);
    } catch (const std::bad_alloc&) {
        return fail(PV_ERR_OOM, "host buffer of %zu elements", n);
    }
    // the callback's 128-bit state: SplitMix64 outputs 1 and 2 of seed_value
    uint64_t state[2];
    for (int j = 0; j < 2; ++j) {
        uint64_t z = seed_value + uint64_t(j + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        state[j] = z ^ (z >> 31);
    }
    size_t e = 0;
    int64_t r[4];
    for (int64_t z = 0; z < l->L[2]; ++z)
        for (int64_t y = 0; y < l->L[1]; ++y)
            for (int64_t x = 0; x < l->L[0]; ++x)
                for (int o = 0; o < l->n_orb; ++o)
                    for (int k = 0; k < nb; ++k, ++e) {
                        r[0] = x;
                        r[1] = y;
                        r[2] = z;
                        r[3] = o;
                        const double re = fnc(r, k, parm, state);
                        const double im = fnc_im ? fnc_im(r, k, parm, state) : 0.0;
                        if (dtype == PV_C128) {
                            h64[2 * e] = re;
                            h64[2 * e + 1] = im;
                        } else {
                            h32[2 * e] = float(re);
                            h32[2 * e + 1] = float(im);
                        }
                    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const void* src = dtype == PV_C128 ? static_cast<const void*>(h64.data()) : static_cast<const void*>(h32.data());
    PV_HIP(hipMemcpyAsync(out, src, n * elem_bytes(dtype), hipMemcpyHostToDevice, s));
    PV_HIP(hipStreamSynchronize(s));
    return PV_OK;
}

extern "C" pv_status pv_random_block(pv_lattice* l, int dtype, int nb, uint64_t seed, int kind, int64_t row0,
                                     void* out, void* stream) {
    if (!l) return fail(PV_ERR_INVALID_ARG, "lattice is NULL");
    pv_status st;
    if (dtype != PV_C128 && dtype != PV_C64) return fail(PV_ERR_INVALID_ARG, "dtype must be PV_C128 or PV_C64");
    if ((st = check_nb(nb)) != PV_OK) return st;
    if (kind != PV_RANDOM_PHASE && kind != PV_RANDOM_Z4)
        return fail(PV_ERR_INVALID_ARG, "kind %d: need PV_RANDOM_PHASE or PV_RANDOM_Z4", kind);
    if (row0 < 0 || row0 > INT64_MAX / nb - l->n_rows)
        return fail(PV_ERR_INVALID_ARG, "row0 = %lld: need 0 <= row0 and (row0 + n_rows) * nb < 2^63",
                    (long long)row0);
    if ((st = check_vec(out, dtype, "out")) != PV_OK) return st;
    int dev;
    if (hipGetDevice(&dev) != hipSuccess) return fail(PV_ERR_NO_DEVICE, "no HIP device");
    PV_HIP(pv::launch_random_block(dtype, kind, l->n_rows * nb, seed, uint64_t(row0) * uint64_t(nb), out,
                                   static_cast<hipStream_t>(stream)));
    return PV_OK;
}

// ---------------------------------------------------------------------------
// Chebyshev series / propagation
// ---------------------------------------------------------------------------
namespace {

// acc/out: Y = sum_k coef_k T_k(H~) X.  The accumulator `acc` is written by
// the first sweep and updated by the later ones; the last sweep writes
// acc + coef_K w_K to `out` (which may be X itself when K >= 2, since X is no
// longer read by then).  W1, W2: two work vectors.
pv_status run_series(pv_lattice* l, int dtype, int nb, double a, double b, int K, const double* coef,
                     const void* X, void* acc, void* out, void* W1, void* W2, hipStream_t s) {
    const int64_t n_elem = l->n_rows * nb;
    if (K == 0) {
        PV_HIP(pv::launch_scale_block(dtype, n_elem, X, coef[0], coef[1], out, s));
        return PV_OK;
    }
    pv::SweepParams p = base_params(l, dtype, nb);
    pv_status st;
    if ((st = fill_traversal(l, dtype, nb, p)) != PV_OK) return st;
    // k = 1
    p.x = X;
    p.y = W1;
    p.z = nullptr;
    p.alpha = 1.0 / a;
    p.beta = b;
    p.gamma = 0.0;
    p.eta0_re = coef[0];
    p.eta0_im = coef[1];
    p.eta_re = coef[2];
    p.eta_im = coef[3];
    p.acc_out = (K == 1) ? out : acc;
    p.ep = pv::EP_ACC_INIT | (K >= 2 ? pv::EP_STORE_Y : 0u);
    PV_HIP(pv::launch_sweep(p, num_cus(), s));
    const void* prev = X;
    void* cur = W1;
    p.alpha = 2.0 / a;
    p.gamma = -1.0;
    for (int k = 2; k <= K; ++k) {
        void* next = (k == 2) ? W2 : const_cast<void*>(prev);
        p.x = cur;
        p.z = prev;
        p.y = next;
        p.eta_re = coef[2 * k];
        p.eta_im = coef[2 * k + 1];
        p.acc_in = acc;
        p.acc_out = (k == K) ? out : acc;
        p.ep = pv::EP_ACC_ADD | (k < K ? pv::EP_STORE_Y : 0u);
        PV_HIP(pv::launch_sweep(p, num_cus(), s));
        prev = cur;
        cur = next;
    }
    return PV_OK;
}

// The same series with w_k written to wbuf(k) for k = 1..K, the last
// included (never in place: every w_k stays readable afterwards).
template <class WB>
pv_status run_series_keep(pv_lattice* l, int dtype, int nb, double a, double b, int K, const double* coef,
                          const void* X, void* acc, void* out, WB&& wbuf, hipStream_t s) {
    pv::SweepParams p = base_params(l, dtype, nb);
    pv_status st;
    if ((st = fill_traversal(l, dtype, nb, p)) != PV_OK) return st;
    p.x = X;
    p.y = wbuf(1);
    p.z = nullptr;
    p.alpha = 1.0 / a;
    p.beta = b;
    p.gamma = 0.0;
    p.eta0_re = coef[0];
    p.eta0_im = coef[1];
    p.eta_re = coef[2];
    p.eta_im = coef[3];
    p.acc_out = (K == 1) ? out : acc;
    p.ep = pv::EP_ACC_INIT | pv::EP_STORE_Y;
    PV_HIP(pv::launch_sweep(p, num_cus(), s));
    p.alpha = 2.0 / a;
    p.gamma = -1.0;
    for (int k = 2; k <= K; ++k) {
        p.x = wbuf(k - 1);
        p.z = k == 2 ? X : wbuf(k - 2);
        p.y = wbuf(k);
        p.eta_re = coef[2 * k];
        p.eta_im = coef[2 * k + 1];
        p.acc_in = acc;
        p.acc_out = (k == K) ? out : acc;
        p.ep = pv::EP_ACC_ADD | pv::EP_STORE_Y;
        PV_HIP(pv::launch_sweep(p, num_cus(), s));
    }
    return PV_OK;
}

pv_status check_series_args(pv_lattice* l, int dtype, int nb, double a, double b) {
    if (!l) return fail(PV_ERR_INVALID_ARG, "lattice is NULL");
    pv_status st;
    if ((st = check_dtype(l, dtype)) != PV_OK) return st;
    if ((st = check_nb(nb)) != PV_OK) return st;
    if (!(a > 0.0) || !std::isfinite(a) || !std::isfinite(b)) return fail(PV_ERR_INVALID_ARG, "need finite a > 0 and b");
    return PV_OK;
}

}  // namespace

extern "C" size_t pv_cheb_series_workspace_size(const pv_lattice* l, int dtype, int nb) {
    if (!l || !is_pow2(nb) || nb > PV_MAX_NB || (dtype != PV_C128 && dtype != PV_C64)) return 0;
    return 2 * vec_bytes(l, dtype, nb);
}

extern "C" pv_status pv_cheb_series(pv_lattice* l, int dtype, int nb, double a, double b, int K, const double* coef,
                                    const void* X, void* Y, void* work, size_t work_bytes, void* stream) {
    pv_status st;
    if ((st = check_series_args(l, dtype, nb, a, b)) != PV_OK) return st;
    if ((st = check_vec(X, dtype, "X")) != PV_OK) return st;
    if ((st = check_vec(Y, dtype, "Y")) != PV_OK) return st;
    if (X == Y) return fail(PV_ERR_INVALID_ARG, "X and Y must differ");
    if (K < 0 || !coef) return fail(PV_ERR_INVALID_ARG, "need K >= 0 and coef[K+1]");
    for (int k = 0; k <= K; ++k)
        if (!std::isfinite(coef[2 * k]) || !std::isfinite(coef[2 * k + 1]))
            return fail(PV_ERR_INVALID_ARG, "non-finite series coefficient %d", k);
    const size_t need = pv_cheb_series_workspace_size(l, dtype, nb);
    if (!work || work_bytes < need) return fail(PV_ERR_WORKSPACE, "workspace %zu < %zu bytes", work_bytes, need);
    if ((st = ensure_device(l)) != PV_OK) return st;
    char* w = static_cast<char*>(work);
    return run_series(l, dtype, nb, a, b, K, coef, X, Y, Y, w, w + vec_bytes(l, dtype, nb),
                      static_cast<hipStream_t>(stream));
}

extern "C" pv_status pv_cheb_tp_coefficients(double a, double dt, int M, double* coef) {
    if (M < 0 || !coef || !std::isfinite(a) || !std::isfinite(dt)) return fail(PV_ERR_INVALID_ARG, "bad arguments");
    std::vector<double> J;
    bessel_j(a * dt, M, J);
    for (int k = 0; k <= M; ++k) {
        // (-i)^k J_k
        const int r = k & 3;
        const double re = (r == 0) ? J[k] : (r == 2 ? -J[k] : 0.0);
        const double im = (r == 1) ? -J[k] : (r == 3 ? J[k] : 0.0);
        coef[2 * k] = re;
        coef[2 * k + 1] = im;
    }
    return PV_OK;
}

extern "C" size_t pv_cheb_propagate_workspace_size(const pv_lattice* l, int dtype, int nb) {
    if (!l || !is_pow2(nb) || nb > PV_MAX_NB || (dtype != PV_C128 && dtype != PV_C64)) return 0;
    return 3 * vec_bytes(l, dtype, nb);
}

extern "C" pv_status pv_cheb_propagate(pv_lattice* l, int dtype, int nb, double a, double b, double dt, int M,
                                       int nsteps, void* psi, void* work, size_t work_bytes, void* stream) {
    pv_status st;
    if ((st = check_series_args(l, dtype, nb, a, b)) != PV_OK) return st;
    if ((st = check_vec(psi, dtype, "psi")) != PV_OK) return st;
    if (M < 1 || nsteps < 0 || !std::isfinite(dt)) return fail(PV_ERR_INVALID_ARG, "need M >= 1, nsteps >= 0");
    const size_t need = pv_cheb_propagate_workspace_size(l, dtype, nb);
    if (!work || work_bytes < need) return fail(PV_ERR_WORKSPACE, "workspace %zu < %zu bytes", work_bytes, need);
    if ((st = ensure_device(l)) != PV_OK) return st;
    std::vector<double> coef(2 * (M + 1));
    pv_cheb_tp_coefficients(a, dt, M, coef.data());
    // eta_0 = e^{-i b dt} c_0, eta_k = 2 e^{-i b dt} c_k
    const std::complex<double> ph = std::exp(std::complex<double>(0.0, -b * dt));
    for (int k = 0; k <= M; ++k) {
        std::complex<double> c(coef[2 * k], coef[2 * k + 1]);
        c *= ph * (k ? 2.0 : 1.0);
        coef[2 * k] = c.real();
        coef[2 * k + 1] = c.imag();
    }
    char* w = static_cast<char*>(work);
    const size_t vb = vec_bytes(l, dtype, nb);
    void* W1 = w;
    void* W2 = w + vb;
    void* ACC = w + 2 * vb;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int step = 0; step < nsteps; ++step) {
        if (M >= 2) {
            if ((st = run_series(l, dtype, nb, a, b, M, coef.data(), psi, ACC, psi, W1, W2, s)) != PV_OK) return st;
        } else {
            if ((st = run_series(l, dtype, nb, a, b, M, coef.data(), psi, ACC, ACC, W1, W2, s)) != PV_OK) return st;
            PV_HIP(pv::launch_copy(ACC, psi, (size_t)l->n_rows * nb * elem_bytes(dtype), s));
        }
    }
    return PV_OK;
}

// ---------------------------------------------------------------------------
// Gram / rotate / copy
// ---------------------------------------------------------------------------
extern "C" size_t pv_gram_workspace_size(int64_t rows, int nx, int ny) {
    if (rows < 0 || nx < 1 || ny < 1 || nx > PV_MAX_NB || ny > PV_MAX_NB) return 0;
    int ncu = num_cus_of_current_device();
    if (ncu <= 0) ncu = 256;
    return align_up((size_t)pv::gram_grid(rows, ncu) * nx * ny * 2 * sizeof(double));
}

extern "C" pv_status pv_gram(int dtype, int64_t rows, int nx, int ny, const void* X, const void* Y, double* G,
                             void* work, size_t work_bytes, void* stream) {
    if (dtype != PV_C128 && dtype != PV_C64) return fail(PV_ERR_INVALID_ARG, "bad dtype");
    if (rows < 1 || nx < 1 || ny < 1 || nx > PV_MAX_NB || ny > PV_MAX_NB)
        return fail(PV_ERR_INVALID_ARG, "need rows >= 1 and 1 <= nx, ny <= %d", PV_MAX_NB);
    pv_status st;
    if ((st = check_vec(X, dtype, "X")) != PV_OK) return st;
    if ((st = check_vec(Y, dtype, "Y")) != PV_OK) return st;
    if (!G) return fail(PV_ERR_INVALID_ARG, "G is NULL");
    const size_t need = pv_gram_workspace_size(rows, nx, ny);
    if (!work || work_bytes < need) return fail(PV_ERR_WORKSPACE, "workspace %zu < %zu bytes", work_bytes, need);
    int ncu = num_cus_of_current_device();
    if (ncu <= 0) return fail(PV_ERR_NO_DEVICE, "no HIP device");
    const int grid = pv::gram_grid(rows, ncu);
    PV_HIP(pv::launch_gram(dtype, rows, nx, ny, X, Y, static_cast<double*>(work), grid, G,
                           static_cast<hipStream_t>(stream)));
    return PV_OK;
}

extern "C" pv_status pv_block_rotate(int dtype, int64_t rows, int nx, int ny, const void* X, const double* Q,
                                     int accumulate, void* Y, void* stream) {
    if (dtype != PV_C128 && dtype != PV_C64) return fail(PV_ERR_INVALID_ARG, "bad dtype");
    if (rows < 1 || nx < 1 || ny < 1 || nx > PV_MAX_NB || ny > PV_MAX_NB)
        return fail(PV_ERR_INVALID_ARG, "need rows >= 1 and 1 <= nx, ny <= %d", PV_MAX_NB);
    pv_status st;
    if ((st = check_vec(X, dtype, "X")) != PV_OK) return st;
    if ((st = check_vec(Y, dtype, "Y")) != PV_OK) return st;
    if (!Q) return fail(PV_ERR_INVALID_ARG, "Q is NULL");
    if (X == Y) return fail(PV_ERR_INVALID_ARG, "X and Y must differ");
    int dev;
    if (hipGetDevice(&dev) != hipSuccess) return fail(PV_ERR_NO_DEVICE, "no HIP device");
    PV_HIP(pv::launch_rotate(dtype, rows, nx, ny, X, Q, accumulate ? 1 : 0, Y, static_cast<hipStream_t>(stream)));
    return PV_OK;
}

extern "C" pv_status pv_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst || bytes % 16 || (reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16)
        return fail(PV_ERR_INVALID_ARG, "copy needs 16-byte aligned pointers and size");
    int dev;
    if (hipGetDevice(&dev) != hipSuccess) return fail(PV_ERR_NO_DEVICE, "no HIP device");
    PV_HIP(pv::launch_copy(src, dst, bytes, static_cast<hipStream_t>(stream)));
    return PV_OK;
}

extern "C" pv_status pv_stream_read(const void* x, size_t bytes, void* sink, void* stream) {
    static_assert(pv::STREAM_READ_GROUPS * 4 * 4 == PV_STREAM_READ_SINK_BYTES, "sink size");
    if (!x || !sink || bytes % 16 || reinterpret_cast<uintptr_t>(x) % 16 || reinterpret_cast<uintptr_t>(sink) % 4)
        return fail(PV_ERR_INVALID_ARG, "read probe needs a 16-byte aligned source and size and a 4-byte aligned sink");
    int dev;
    if (hipGetDevice(&dev) != hipSuccess) return fail(PV_ERR_NO_DEVICE, "no HIP device");
    PV_HIP(pv::launch_read(x, bytes, sink, static_cast<hipStream_t>(stream)));
    return PV_OK;
}

extern "C" pv_status pv_stream_triad(const void* x, const void* z, void* y, size_t bytes, void* stream) {
    if (!x || !z || !y || bytes % 16 ||
        (reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(z) | reinterpret_cast<uintptr_t>(y)) % 16)
        return fail(PV_ERR_INVALID_ARG, "triad needs 16-byte aligned pointers and size");
    int dev;
    if (hipGetDevice(&dev) != hipSuccess) return fail(PV_ERR_NO_DEVICE, "no HIP device");
    PV_HIP(pv::launch_triad(x, z, y, bytes, static_cast<hipStream_t>(stream)));
    return PV_OK;
}

// ---------------------------------------------------------------------------
// Launch shapes and the autotuner
// ---------------------------------------------------------------------------
namespace {

pv_status check_tuning(int dtype, const pv_tuning& t) {
    if (t.kernel < 0 || t.kernel > 2) return fail(PV_ERR_INVALID_ARG, "tuning.kernel = %d (0, 1 or 2)", t.kernel);
    const int e = t.elems_per_lane;
    if (e != 0 && (dtype == PV_C128 ? (e != 1 && e != 2) : (e != 2 && e != 4)))
        return fail(PV_ERR_INVALID_ARG, "tuning.elems_per_lane = %d not available for this dtype", e);
    if (t.walk_planes < 0 || t.strip_rows < 0 || t.slab_rows < 0)
        return fail(PV_ERR_INVALID_ARG, "tuning: negative walk_planes, strip_rows or slab_rows");
    if (t.groups_per_xcd < 0 || t.groups_per_xcd > 256)
        return fail(PV_ERR_INVALID_ARG, "tuning.groups_per_xcd = %d (0..256)", t.groups_per_xcd);
    if (t.tiles_per_group < 0 || t.tiles_per_group > 64)
        return fail(PV_ERR_INVALID_ARG, "tuning.tiles_per_group = %d (0..64)", t.tiles_per_group);
    if (t.workgroup_size != 0 && t.workgroup_size != 256 && t.workgroup_size != 512)
        return fail(PV_ERR_INVALID_ARG, "tuning.workgroup_size = %d (0, 256 or 512)", t.workgroup_size);
    return PV_OK;
}

std::string tune_key(const pv_lattice* l, int dtype, int nb) {
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        cus = prop.multiProcessorCount;
    }
    // generic stencils: their offsets, and the generated kernels' pattern when
    // sweeps use them (FNV-1a)
    unsigned long long gh = 0;
    if (l->family == pv::FAM_GENERIC) {
        gh = 14695981039346656037ull;
        auto mix = [&](const void* data, size_t n) {
            for (size_t i = 0; i < n; ++i) {
                gh ^= static_cast<const unsigned char*>(data)[i];
                gh *= 1099511628211ull;
            }
        };
        mix(l->offsets.data(), l->offsets.size() * sizeof(int));
        if (uses_codegen(l)) mix(l->cg_src.data(), l->cg_src.size());
    }
    char buf[512];
    std::snprintf(buf, sizeof buf,
                  "family=%d orb=%d L=%lldx%lldx%lld bc=%d%d%d nb=%d dtype=%d vtype=%d dev=%s cus=%d stencil=%016llx",
                  l->family, l->n_orb, (long long)l->L[0], (long long)l->L[1], (long long)l->L[2], l->periodic[0],
                  l->periodic[1], l->periodic[2], nb, dtype, l->rng_on ? 2 : (l->V ? l->vtype : -1), arch.c_str(), cus,
                  gh);
    return buf;
}

constexpr int kNumTuneFields = 8;
const char* const kTuneFields[kNumTuneFields] = {"kernel",         "elems_per_lane",  "walk_planes", "strip_rows",
                                                 "groups_per_xcd", "tiles_per_group", "slab_rows",   "workgroup_size"};

int* tune_field(pv_tuning& t, int i) {
    int* f[kNumTuneFields] = {&t.kernel,         &t.elems_per_lane,  &t.walk_planes, &t.strip_rows,
                              &t.groups_per_xcd, &t.tiles_per_group, &t.slab_rows,   &t.workgroup_size};
    return f[i];
}

// Cache lines: {"key": "...", "kernel": k, ..., "acc_kernel": k, ..., "ms": t}
// (the Chebyshev-step shape, then the series-step shape).  Returns true and
// fills t, ta for the last line whose key matches and that holds both.
bool cache_lookup(const char* path, const std::string& key, pv_tuning& t, pv_tuning& ta) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    bool found = false;
    char line[4096];
    const std::string want = "\"key\": \"" + key + "\"";
    while (std::fgets(line, sizeof line, f)) {
        if (!std::strstr(line, want.c_str())) continue;
        pv_tuning r[2] = {};
        bool ok = true;
        for (int h = 0; h < 2 && ok; ++h)
            for (int i = 0; i < kNumTuneFields && ok; ++i) {
                const std::string name = std::string("\"") + (h ? "acc_" : "") + kTuneFields[i] + "\": ";
                const char* q = std::strstr(line, name.c_str());
                if (!q) { ok = false; break; }
                *tune_field(r[h], i) = int(std::strtol(q + name.size(), nullptr, 10));
            }
        if (ok) {
            t = r[0];
            ta = r[1];
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_append(const char* path, const std::string& key, const pv_tuning& t, const pv_tuning& ta, double ms) {
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "{\"key\": \"%s\"", key.c_str());
    pv_tuning c[2] = {t, ta};
    for (int h = 0; h < 2; ++h)
        for (int i = 0; i < kNumTuneFields; ++i)
            std::fprintf(f, ", \"%s%s\": %d", h ? "acc_" : "", kTuneFields[i], *tune_field(c[h], i));
    std::fprintf(f, ", \"ms\": %.6f}\n", ms);
    std::fclose(f);
}

}  // namespace

extern "C" pv_status pv_lattice_set_tuning(pv_lattice* l, int dtype, int nb, const pv_tuning* t) {
    if (!l) return fail(PV_ERR_INVALID_ARG, "lattice is NULL");
    pv_status st;
    if (dtype != PV_C128 && dtype != PV_C64) return fail(PV_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    if ((st = check_nb(nb)) != PV_OK) return st;
    pv_tuning z{};
    if (t && (st = check_tuning(dtype, *t)) != PV_OK) return st;
    l->tune[dtype == PV_C128 ? 0 : 1][log2_nb(nb)] = t ? *t : z;
    l->tune_acc[dtype == PV_C128 ? 0 : 1][log2_nb(nb)] = z;   // series steps follow the set shape
    return PV_OK;
}

extern "C" pv_status pv_lattice_get_tuning(const pv_lattice* l, int dtype, int nb, pv_tuning* t) {
    if (!l || !t) return fail(PV_ERR_INVALID_ARG, "lattice or output is NULL");
    pv_status st;
    if (dtype != PV_C128 && dtype != PV_C64) return fail(PV_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    if ((st = check_nb(nb)) != PV_OK) return st;
    *t = l->tune[dtype == PV_C128 ? 0 : 1][log2_nb(nb)];
    return PV_OK;
}

extern "C" pv_status pv_lattice_set_codegen(pv_lattice* l, int enable) {
    if (!l) return fail(PV_ERR_INVALID_ARG, "lattice is NULL");
    if (enable != 0 && enable != 1) return fail(PV_ERR_INVALID_ARG, "enable must be 0 or 1");
    l->codegen = enable;
    return PV_OK;
}

extern "C" pv_status pv_lattice_get_codegen(const pv_lattice* l, int* active) {
    if (!l || !active) return fail(PV_ERR_INVALID_ARG, "lattice or output is NULL");
    *active = uses_codegen(l) ? 1 : 0;
    return PV_OK;
}

extern "C" int pv_codegen_instances(void) { return pv::codegen_instances(); }

extern "C" pv_status pv_lattice_codegen_source(const pv_lattice* l, char* buf, size_t len, size_t* needed) {
    if (!l) return fail(PV_ERR_INVALID_ARG, "lattice is NULL");
    if (l->family != pv::FAM_GENERIC)
        return fail(PV_ERR_UNSUPPORTED, "the stencil is a built-in family (family %d): no generated pattern", l->family);
    if (l->cg_src.empty())
        return fail(PV_ERR_UNSUPPORTED, "the stencil's rows need more than %d slots: no generated pattern",
                    pv::MAX_SLOTS_K);
    if (needed) *needed = l->cg_src.size() + 1;
    if (buf && len) {
        const size_t n = std::min(len - 1, l->cg_src.size());
        std::memcpy(buf, l->cg_src.data(), n);
        buf[n] = '\0';
    }
    return PV_OK;
}

extern "C" size_t pv_autotune_workspace_size(const pv_lattice* l, int dtype, int nb) {
    if (!l || !is_pow2(nb) || nb > PV_MAX_NB || (dtype != PV_C128 && dtype != PV_C64)) return 0;
    return 3 * vec_bytes(l, dtype, nb) + partial_bytes(l, nb) + align_up(sizeof(double) * 4 * nb);
}

extern "C" pv_status pv_autotune(pv_lattice* l, int dtype, int nb, const char* cache_path, void* work,
                                 size_t work_bytes, void* stream, pv_tuning* out, double* ms_out) {
    if (!l) return fail(PV_ERR_INVALID_ARG, "lattice is NULL");
    pv_status st;
    if ((st = check_dtype(l, dtype)) != PV_OK) return st;
    if ((st = check_nb(nb)) != PV_OK) return st;
    const size_t need = pv_autotune_workspace_size(l, dtype, nb);
    if (!work || work_bytes < need) return fail(PV_ERR_WORKSPACE, "workspace %zu < %zu bytes", work_bytes, need);
    if ((st = ensure_device(l)) != PV_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!cache_path) cache_path = std::getenv("PV_TUNE_CACHE");
    const std::string key = tune_key(l, dtype, nb);
    const int di = dtype == PV_C128 ? 0 : 1, ni = log2_nb(nb);
    pv_tuning& slot = l->tune[di][ni];
    pv_tuning& slot_acc = l->tune_acc[di][ni];
    {
        pv_tuning c{}, ca{};
        if (cache_path && cache_lookup(cache_path, key, c, ca) && check_tuning(dtype, c) == PV_OK &&
            check_tuning(dtype, ca) == PV_OK) {
            slot = c;
            slot_acc = ca;
            if (out) *out = c;
            if (ms_out) *ms_out = 0.0;
            return PV_OK;
        }
    }

    // buffers: x = y = acc = 0; the Chebyshev step y = 2 H~ x - y with fused
    // dots, and the series step y = 2 H~ x - y, acc += eta y
    char* w = static_cast<char*>(work);
    const size_t vb = vec_bytes(l, dtype, nb);
    void* x = w;
    void* y = w + vb;
    void* acc = w + 2 * vb;
    double* part = reinterpret_cast<double*>(w + 3 * vb);
    double* dots = reinterpret_cast<double*>(w + 3 * vb + partial_bytes(l, nb));
    PV_HIP(pv::launch_zero(w, 3 * vb, s));
    hipEvent_t e0, e1;
    PV_HIP(hipEventCreate(&e0));
    PV_HIP(hipEventCreate(&e1));
    const pv_tuning saved = slot, saved_acc = slot_acc;
    bool series = false;   // which step the candidates are timed on
    auto run = [&](int reps) -> hipError_t {
        for (int r = 0; r < reps; ++r) {
            pv::SweepParams p = base_params(l, dtype, nb);
            fill_traversal(l, dtype, nb, p);
            p.x = x; p.z = y; p.y = y;
            p.alpha = 2.0 / 8.0; p.beta = 0.0; p.gamma = -1.0;
            if (series) {
                p.ep = pv::EP_STORE_Y | pv::EP_ACC_ADD;
                p.acc_in = acc;
                p.acc_out = acc;
                p.eta_re = 0.5;
                p.eta_im = 0.25;
                if (hipError_t e = pv::launch_sweep(p, num_cus(), s); e != hipSuccess) return e;
            } else {
                p.ep = pv::EP_STORE_Y | pv::EP_DOTS;
                p.partials = part;
                hipError_t e = pv::launch_sweep(p, num_cus(), s);
                if (e == hipSuccess) e = pv::launch_reduce_dots(part, p.grid, nb, 0, dots, 0, 0, 0.0, s);
                if (e != hipSuccess) return e;
            }
        }
        return hipSuccess;
    };
    // time of one step under shape t (milliseconds): warm-up first, then the
    // fastest of three batches of about 10 ms each (a single short batch lets
    // clock and co-tenant noise pick a shape that moves more bytes)
    auto measure = [&](const pv_tuning& t, double& ms) -> hipError_t {
        (series ? slot_acc : slot) = t;
        hipError_t e = run(1);
        if (e != hipSuccess) return e;
        if ((e = hipEventRecord(e0, s)) != hipSuccess) return e;
        if ((e = run(1)) != hipSuccess) return e;
        if ((e = hipEventRecord(e1, s)) != hipSuccess) return e;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
        float t1 = 0.f;
        if ((e = hipEventElapsedTime(&t1, e0, e1)) != hipSuccess) return e;
        int reps = t1 > 0.f ? int(10.0 / t1) : 10;
        reps = reps < 2 ? 2 : (reps > 50 ? 50 : reps);
        ms = 1e300;
        for (int b = 0; b < 3; ++b) {
            if ((e = hipEventRecord(e0, s)) != hipSuccess) return e;
            if ((e = run(reps)) != hipSuccess) return e;
            if ((e = hipEventRecord(e1, s)) != hipSuccess) return e;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
            float tt = 0.f;
            if ((e = hipEventElapsedTime(&tt, e0, e1)) != hipSuccess) return e;
            if (double(tt) / reps < ms) ms = double(tt) / reps;
        }
        return hipSuccess;
    };
    hipError_t herr = hipSuccess;
    const bool cg = uses_codegen(l);
    const bool compiled = l->family != pv::FAM_GENERIC || generic_stageable(l) || cg;
    const int lw = int(l->dim == 3 ? l->L[2] : l->L[1]);
    // coordinate search: 1. kernel, elements per lane and lanes per workgroup
    // at default shapes;
    // for the staged winner 2. strip height, 3. planes per walk, 4. workgroups
    // per XCD; for the direct winner, tiles per workgroup
    auto search = [&](pv_tuning& best, double& best_ms) {
        best = pv_tuning{};
        best_ms = 1e300;
        // a candidate must beat the incumbent by 1% (timing noise would
        // otherwise flip between near-equal shapes from run to run), plus
        // `extra`, the fraction of the step's bytes it moves on top
        auto consider = [&](const pv_tuning& t, double extra = 0.0) {
            if (herr != hipSuccess) return;
            double ms = 0;
            herr = measure(t, ms);
            if (herr == hipSuccess && ms < (0.99 - extra) * best_ms) {
                best_ms = ms;
                best = t;
            }
        };
        pv_tuning t{};
        t.kernel = 1;
        consider(t);
        if (compiled) {
            // elements per lane x lanes per workgroup (512 only for compiled families)
            const int es[2] = {dtype == PV_C128 ? 1 : 2, dtype == PV_C128 ? 2 : 4};
            for (int wg : {256, 512})
                for (int e : es) {
                    if (wg == 512 && l->family == pv::FAM_GENERIC && !cg) continue;
                    t = pv_tuning{};
                    t.kernel = 2;
                    t.elems_per_lane = e;
                    t.workgroup_size = wg == 512 ? 512 : 0;
                    consider(t);
                }
        }
        if (best.kernel == 2) {
            for (int v : {4, 8, 16, 32, 64}) { t = best; t.strip_rows = v; consider(t); }
            // a walk of v planes re-reads two ring rows that a whole walk
            // reads once per lw planes: x is one of about three streams
            for (int v : {8, 16, 32})
                if (v < lw) {
                    t = best;
                    t.walk_planes = v;
                    consider(t, (2.0 / v - 2.0 / lw) / 3.0);
                }
            for (int v : {32, 64, 96, 128}) { t = best; t.groups_per_xcd = v; consider(t); }
        } else {
            for (int v : {32, 64}) { t = best; t.tiles_per_group = v; consider(t); }
        }
    };
    pv_tuning best{}, best_acc{};
    double best_ms = 0.0, best_acc_ms = 0.0;
    search(best, best_ms);
    if (herr == hipSuccess) {
        slot = best;
        series = true;
        search(best_acc, best_acc_ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (herr != hipSuccess) {
        slot = saved;
        slot_acc = saved_acc;
        return hip_fail(herr, "autotune");
    }
    slot = best;
    slot_acc = best_acc;
    if (cache_path) cache_append(cache_path, key, best, best_acc, best_ms);
    if (out) *out = best;
    if (ms_out) *ms_out = best_ms;
    return PV_OK;
}

// ---------------------------------------------------------------------------
// Chebyshev filter diagonalisation (Sec. 4.2)
// ---------------------------------------------------------------------------
#include "pv_dense.hpp"

extern "C" pv_status pv_host_heev(int n, const double* A, double* w, double* V) {
    if (n < 1 || !A || !w || !V) return fail(PV_ERR_INVALID_ARG, "pv_host_heev: bad arguments");
    std::vector<pvd::cd> M((size_t)n * n), U;
    for (size_t i = 0; i < M.size(); ++i) M[i] = pvd::cd(A[2 * i], A[2 * i + 1]);
    std::vector<double> ev;
    pvd::heev_jacobi(n, M, ev, U);
    for (int i = 0; i < n; ++i) w[i] = ev[i];
    for (size_t i = 0; i < U.size(); ++i) {
        V[2 * i] = U[i].real();
        V[2 * i + 1] = U[i].imag();
    }
    return PV_OK;
}

extern "C" pv_status pv_chebfd_filter_coefficients(double lam_l, double lam_r, double a, double b, int K,
                                                   double* coef) {
    if (K < 0 || !coef || !(a > 0.0)) return fail(PV_ERR_INVALID_ARG, "bad filter arguments");
    const double xl = (lam_l - b) / a, xr = (lam_r - b) / a;
    if (!(xl >= -1.0 && xl < xr && xr <= 1.0)) return fail(PV_ERR_INVALID_ARG, "window must lie inside the scaled spectrum");
    const double al = std::acos(xl), ar = std::acos(xr);
    // Jackson damping with N = K + 1 terms (Weisse et al. 2006), Chebyshev
    // series of the window indicator
    const int N = K + 1;
    const double q = M_PI / (N + 1);
    for (int k = 0; k <= K; ++k) {
        const double g = ((N - k + 1) * std::cos(q * k) + std::sin(q * k) / std::tan(q)) / (N + 1);
        const double c = (k == 0) ? (al - ar) / M_PI : 2.0 * (std::sin(k * al) - std::sin(k * ar)) / (k * M_PI);
        coef[k] = g * c;
    }
    return PV_OK;
}

namespace {

struct FdLayout {
    size_t vb;      // bytes of one [rows][bw] block
    size_t Y, W, S1, S2, gp, sp, G, D;
    size_t total;
    int groups;     // row-chunk groups of the block Gram
};

FdLayout fd_layout(const pv_lattice* l, int dtype, int bw, int nblk) {
    FdLayout L{};
    L.vb = vec_bytes(l, dtype, bw);
    size_t off = 0;
    L.Y = off; off += L.vb * nblk;
    L.W = off; off += L.vb * nblk;
    L.S1 = off; off += L.vb;
    L.S2 = off; off += L.vb;
    int ncu = num_cus_of_current_device();
    if (ncu <= 0) ncu = 256;
    L.groups = pv::block_gram_groups(l->n_rows, nblk, ncu);
    L.gp = off; off += align_up((size_t)nblk * nblk * L.groups * bw * bw * 2 * sizeof(double));
    L.sp = off; off += pv_spmmv_workspace_size(l, dtype, bw);
    const size_t ns = (size_t)bw * nblk;
    L.G = off; off += align_up(ns * ns * 2 * sizeof(double));
    L.D = off; off += align_up(ns * 4 * sizeof(double));
    L.total = off;
    return L;
}

}  // namespace

extern "C" size_t pv_chebfd_workspace_size(const pv_lattice* l, int dtype, int bw, int nblk) {
    if (!l || !is_pow2(bw) || bw > PV_MAX_NB || nblk < 1 || (dtype != PV_C128 && dtype != PV_C64)) return 0;
    return fd_layout(l, dtype, bw, nblk).total;
}

extern "C" pv_status pv_chebfd(pv_lattice* l, int dtype, int bw, int nblk, double a, double b, double lam_l,
                               double lam_r, int degree, int n_target, double tol, int max_iter, void* X,
                               double* theta, double* res, int* n_conv, int* iters, void* work, size_t work_bytes,
                               void* stream) {
    pv_status st;
    if ((st = check_series_args(l, dtype, bw, a, b)) != PV_OK) return st;
    if ((st = check_vec(X, dtype, "X")) != PV_OK) return st;
    const int ns = bw * nblk;
    if (nblk < 1 || ns > 1024) return fail(PV_ERR_INVALID_ARG, "need 1 <= bw*nblk <= 1024");
    if (degree < 1 || n_target < 1 || n_target > ns || !(tol > 0.0) || max_iter < 1)
        return fail(PV_ERR_INVALID_ARG, "need degree >= 1, 1 <= n_target <= bw*nblk, tol > 0, max_iter >= 1");
    if (!theta || !res || !n_conv || !iters) return fail(PV_ERR_INVALID_ARG, "NULL output");
    std::vector<double> fc(degree + 1);
    if ((st = pv_chebfd_filter_coefficients(lam_l, lam_r, a, b, degree, fc.data())) != PV_OK) return st;
    const FdLayout Lw = fd_layout(l, dtype, bw, nblk);
    if (!work || work_bytes < Lw.total) return fail(PV_ERR_WORKSPACE, "workspace %zu < %zu bytes", work_bytes, Lw.total);
    if ((st = ensure_device(l)) != PV_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(work);
    char* Xc = static_cast<char*>(X);
    auto blk = [&](char* base, int i) { return static_cast<void*>(base + Lw.vb * i); };
    char* Yb = w + Lw.Y;
    char* Wb = w + Lw.W;
    double* Gd = reinterpret_cast<double*>(w + Lw.G);
    double* Dd = reinterpret_cast<double*>(w + Lw.D);
    const int64_t rows = l->n_rows;
    std::vector<double> coef(2 * (degree + 1), 0.0);
    for (int k = 0; k <= degree; ++k) coef[2 * k] = fc[k];
    const double centre = 0.5 * (lam_l + lam_r);
    std::vector<double> Gh((size_t)ns * ns * 2);

    // G = A^H B over the whole search space (A, B as nblk blocks) in one
    // pass, then to the host: one synchronisation per Gram
    const int64_t bstride = int64_t(Lw.vb / elem_bytes(dtype));
    auto block_gram = [&](char* A, char* B, bool hermitian) -> pv_status {
        PV_HIP(pv::launch_block_gram(dtype, rows, bw, nblk, A, B, bstride, hermitian ? 1 : 0,
                                     reinterpret_cast<double*>(w + Lw.gp), Lw.groups, Gd, s));
        PV_HIP(hipMemcpyAsync(Gh.data(), Gd, Gh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        PV_HIP(hipStreamSynchronize(s));
        for (double v : Gh)
            if (!std::isfinite(v))
                return fail(PV_ERR_NONFINITE, "search space holds non-finite values (start block or field)");
        return PV_OK;
    };
    // OUT_j = sum_i IN_i M_ij for an ns x ns host matrix M: one upload, one
    // launch over every output block
    std::vector<double> Mh((size_t)ns * ns * 2);
    auto block_rotate = [&](char* IN, const std::vector<pvd::cd>& M, char* OUT) -> pv_status {
        for (size_t k = 0; k < M.size(); ++k) {
            Mh[2 * k] = M[k].real();
            Mh[2 * k + 1] = M[k].imag();
        }
        PV_HIP(hipMemcpyAsync(Gd, Mh.data(), Mh.size() * sizeof(double), hipMemcpyHostToDevice, s));
        PV_HIP(pv::launch_block_rotate(dtype, rows, bw, nblk, nblk, IN, bstride, Gd, OUT, bstride, s));
        PV_HIP(hipStreamSynchronize(s));   // Mh is rewritten by the next rotation
        return PV_OK;
    };
    auto host_matrix = [&]() {
        std::vector<pvd::cd> M((size_t)ns * ns);
        for (size_t i = 0; i < M.size(); ++i) M[i] = pvd::cd(Gh[2 * i], Gh[2 * i + 1]);
        return M;
    };

    std::vector<double> th(ns), rr(ns);
    std::vector<int> order(ns);
    int it = 0;
    bool converged = false;
    for (it = 1; it <= max_iter; ++it) {
        // 1. filter every block: Y_b = p(H~) X_b
        for (int bb = 0; bb < nblk; ++bb)
            if ((st = run_series(l, dtype, bw, a, b, degree, coef.data(), blk(Xc, bb), blk(Yb, bb), blk(Yb, bb),
                                 w + Lw.S1, w + Lw.S2, s)) != PV_OK)
                return st;
        // 2. orthonormalise: Cholesky QR, twice (Y <-> W)
        char* cur = Yb;
        char* oth = Wb;
        for (int pass = 0; pass < 2; ++pass) {
            if ((st = block_gram(cur, cur, true)) != PV_OK) return st;
            std::vector<pvd::cd> R = host_matrix(), Minv;
            if (!pvd::cholesky_upper(ns, R))
                return fail(PV_ERR_NOT_CONVERGED, "filtered block lost rank (Cholesky failed) in iteration %d", it);
            pvd::invert_upper(ns, R, Minv);
            if ((st = block_rotate(cur, Minv, oth)) != PV_OK) return st;
            std::swap(cur, oth);
        }
        // cur = Q (orthonormal), oth = scratch
        // 3. Rayleigh-Ritz: H Q into oth, H_S = Q^H H Q
        {
            const std::vector<double> one(bw, 1.0), zero(bw, 0.0);
            for (int bb = 0; bb < nblk; ++bb)
                if ((st = pv_spmmv(l, dtype, bw, blk(cur, bb), nullptr, blk(oth, bb), one.data(), zero.data(),
                                   zero.data(), 0, nullptr, w + Lw.sp, pv_spmmv_workspace_size(l, dtype, bw),
                                   stream)) != PV_OK)
                    return st;
        }
        if ((st = block_gram(cur, oth, false)) != PV_OK) return st;
        std::vector<pvd::cd> Hs = host_matrix(), U;
        for (int i = 0; i < ns; ++i)
            for (int j = i + 1; j < ns; ++j) {
                const pvd::cd m = 0.5 * (Hs[(size_t)i * ns + j] + std::conj(Hs[(size_t)j * ns + i]));
                Hs[(size_t)i * ns + j] = m;
                Hs[(size_t)j * ns + i] = std::conj(m);
            }
        std::vector<double> ev;
        pvd::heev_jacobi(ns, Hs, ev, U);
        // order Ritz pairs by distance from the window centre
        for (int i = 0; i < ns; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(),
                         [&](int i, int j) { return std::fabs(ev[i] - centre) < std::fabs(ev[j] - centre); });
        std::vector<pvd::cd> Uo((size_t)ns * ns);
        for (int r = 0; r < ns; ++r)
            for (int c = 0; c < ns; ++c) Uo[(size_t)r * ns + c] = U[(size_t)r * ns + order[c]];
        for (int c = 0; c < ns; ++c) th[c] = ev[order[c]];
        // 4. Ritz vectors into X
        if ((st = block_rotate(cur, Uo, Xc)) != PV_OK) return st;
        // 5. residuals ||H q - theta q|| with per-column shifts and the fused
        // <y,y>, every block, then one copy to the host
        for (int bb = 0; bb < nblk; ++bb) {
            const std::vector<double> one(bw, 1.0), zero(bw, 0.0);
            std::vector<double> sh(th.begin() + bb * bw, th.begin() + (bb + 1) * bw);
            if ((st = pv_spmmv(l, dtype, bw, blk(Xc, bb), nullptr, blk(oth, bb), one.data(), sh.data(), zero.data(),
                               PV_DOT_YY, Dd + (size_t)bb * bw * 4, w + Lw.sp, pv_spmmv_workspace_size(l, dtype, bw),
                               stream)) != PV_OK)
                return st;
        }
        {
            std::vector<double> d((size_t)ns * 4);
            PV_HIP(hipMemcpyAsync(d.data(), Dd, d.size() * sizeof(double), hipMemcpyDeviceToHost, s));
            PV_HIP(hipStreamSynchronize(s));
            for (int c = 0; c < ns; ++c) rr[c] = std::sqrt(std::max(d[c * 4 + 3], 0.0));
        }
        // converged pairs: value in the window, residual <= tol (Ritz values
        // of an oversized search space that belong to no eigenvector keep
        // residuals of order one and never count)
        int count = 0;
        for (int i = 0; i < ns; ++i)
            if (th[i] >= lam_l && th[i] <= lam_r && rr[i] <= tol) ++count;
        converged = count >= n_target;
        if (converged || it == max_iter) break;
    }
    if (it > max_iter) it = max_iter;
    // converged pairs first, each group by distance from the centre (the
    // columns already are): permute X to match
    std::vector<int> perm(ns);
    {
        int k = 0;
        for (int i = 0; i < ns; ++i)
            if (th[i] >= lam_l && th[i] <= lam_r && rr[i] <= tol) perm[k++] = i;
        for (int i = 0; i < ns; ++i)
            if (!(th[i] >= lam_l && th[i] <= lam_r && rr[i] <= tol)) perm[k++] = i;
    }
    bool identity = true;
    for (int i = 0; i < ns; ++i) identity = identity && perm[i] == i;
    if (!identity) {
        std::vector<pvd::cd> P((size_t)ns * ns, pvd::cd(0.0, 0.0));
        for (int c = 0; c < ns; ++c) P[(size_t)perm[c] * ns + c] = 1.0;
        char* tmp = Xc == Yb ? Wb : Yb;
        if ((st = block_rotate(Xc, P, tmp)) != PV_OK) return st;
        PV_HIP(pv::launch_copy(tmp, Xc, Lw.vb * nblk, s));
        PV_HIP(hipStreamSynchronize(s));
    }
    int nc = 0;
    for (int i = 0; i < ns; ++i) {
        theta[i] = th[perm[i]];
        res[i] = rr[perm[i]];
        if (i < n_target && theta[i] >= lam_l && theta[i] <= lam_r && res[i] <= tol) ++nc;
    }
    *n_conv = nc;
    *iters = it;
    if (!converged) return fail(PV_ERR_NOT_CONVERGED, "%d of %d target pairs converged after %d iterations", nc, n_target, it);
    return PV_OK;
}

// ---------------------------------------------------------------------------
// Thick-restart Lanczos with polynomial filtering (trLanczosFD, Sec. 4.2; the
// method of Li, Xi, Vecharynski, Yang and Saad, SIAM J. Sci. Comput. 2016)
// ---------------------------------------------------------------------------
extern "C" pv_status pv_trlanczos_filter(double lam_l, double lam_r, double a, double b, int K, double* coef,
                                         double* tau) {
    if (K < 1 || !coef || !tau || !(a > 0.0)) return fail(PV_ERR_INVALID_ARG, "bad filter arguments");
    const double xl = (lam_l - b) / a, xr = (lam_r - b) / a;
    if (!(xl > -1.0 && xl < xr && xr < 1.0)) return fail(PV_ERR_INVALID_ARG, "window must lie inside the scaled spectrum");
    const double xc = 0.5 * (xl + xr), tc = std::acos(xc);
    // Jackson-damped Chebyshev expansion of a delta peak at xc (N = K + 1 terms)
    const int N = K + 1;
    const double q = M_PI / (N + 1);
    for (int k = 0; k <= K; ++k) {
        const double g = ((N - k + 1) * std::cos(q * k) + std::sin(q * k) / std::tan(q)) / (N + 1);
        coef[k] = g * (k == 0 ? 1.0 : 2.0) * std::cos(k * tc);
    }
    auto eval = [&](double x) {
        double t0 = 1.0, t1 = x, acc = coef[0] + coef[1] * x;
        for (int k = 2; k <= K; ++k) {
            const double t2 = 2.0 * x * t1 - t0;
            acc += coef[k] * t2;
            t0 = t1;
            t1 = t2;
        }
        return acc;
    };
    const double pc = eval(xc);
    if (!(pc > 0.0)) return fail(PV_ERR_INVALID_ARG, "degenerate filter");
    for (int k = 0; k <= K; ++k) coef[k] /= pc;
    *tau = std::min(eval(xl), eval(xr));
    return PV_OK;
}

namespace {

constexpr int kTrBw = 32;   // columns per basis block

struct TrLayout {
    int nblk;
    size_t vbl, vbw;
    size_t V, U, HU, S0, Wv, T1, S1, S2, gp, sp, h, D, total;
};

TrLayout tr_layout(const pv_lattice* l, int dtype, int nbl, int m) {
    TrLayout L{};
    L.nblk = (m + nbl + kTrBw - 1) / kTrBw;
    L.vbl = vec_bytes(l, dtype, nbl);
    L.vbw = vec_bytes(l, dtype, kTrBw);
    size_t off = 0;
    L.V = off; off += L.vbw * L.nblk;
    L.U = off; off += L.vbw * L.nblk;
    L.HU = off; off += L.vbw;
    L.S0 = off; off += L.vbl;
    L.Wv = off; off += L.vbl;
    L.T1 = off; off += L.vbl;
    L.S1 = off; off += L.vbl;
    L.S2 = off; off += L.vbl;
    L.gp = off; off += pv_gram_workspace_size(l->n_rows, kTrBw, kTrBw);
    L.sp = off; off += pv_spmmv_workspace_size(l, dtype, kTrBw);
    L.h = off; off += align_up((size_t)kTrBw * kTrBw * 2 * sizeof(double));
    L.D = off; off += align_up((size_t)kTrBw * 4 * sizeof(double));
    L.total = off;
    return L;
}

bool tr_shape_ok(int nbl, int m) {
    return is_pow2(nbl) && nbl <= kTrBw && m % nbl == 0 && m >= 2 * nbl && m + nbl <= 1024;
}

}  // namespace

extern "C" size_t pv_trlanczos_workspace_size(const pv_lattice* l, int dtype, int nbl, int m) {
    if (!l || !tr_shape_ok(nbl, m) || (dtype != PV_C128 && dtype != PV_C64)) return 0;
    return tr_layout(l, dtype, nbl, m).total;
}

extern "C" pv_status pv_trlanczos_fd(pv_lattice* l, int dtype, double a, double b, double lam_l, double lam_r,
                                     int degree, int nbl, int m, double tol, int max_restarts, const void* v0,
                                     int n_out, void* X, double* theta, double* res, int* n_found, int* restarts,
                                     void* work, size_t work_bytes, void* stream) {
    pv_status st;
    if (!tr_shape_ok(nbl, m))
        return fail(PV_ERR_INVALID_ARG, "need nbl a power of two <= %d, m a multiple of nbl, 2 nbl <= m, m + nbl <= 1024",
                    kTrBw);
    if ((st = check_series_args(l, dtype, nbl, a, b)) != PV_OK) return st;
    if ((st = check_vec(v0, dtype, "v0")) != PV_OK) return st;
    if (degree < 1 || !(tol > 0.0) || max_restarts < 1)
        return fail(PV_ERR_INVALID_ARG, "need degree >= 1, tol > 0, max_restarts >= 1");
    if (n_out < 0 || (n_out > 0 && (!is_pow2(n_out) || n_out > PV_MAX_NB)))
        return fail(PV_ERR_INVALID_ARG, "n_out must be 0 or a power of two <= %d", PV_MAX_NB);
    if (n_out > 0 && (st = check_vec(X, dtype, "X")) != PV_OK) return st;
    if (!theta || !res || !n_found || !restarts) return fail(PV_ERR_INVALID_ARG, "NULL output");
    std::vector<double> fc(degree + 1);
    double tau = 0.0;
    if ((st = pv_trlanczos_filter(lam_l, lam_r, a, b, degree, fc.data(), &tau)) != PV_OK) return st;
    const TrLayout Lw = tr_layout(l, dtype, nbl, m);
    if (!work || work_bytes < Lw.total) return fail(PV_ERR_WORKSPACE, "workspace %zu < %zu bytes", work_bytes, Lw.total);
    if ((st = ensure_device(l)) != PV_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(work);
    const int64_t rows = l->n_rows;
    auto vblk = [&](size_t base, int i) { return static_cast<void*>(w + base + Lw.vbw * i); };
    void* S0 = w + Lw.S0;
    void* Wv = w + Lw.Wv;
    void* T1 = w + Lw.T1;
    double* hd = reinterpret_cast<double*>(w + Lw.h);
    double* Dd = reinterpret_cast<double*>(w + Lw.D);
    const size_t gp_bytes = Lw.sp - Lw.gp;
    std::vector<double> coef(2 * (degree + 1), 0.0);
    for (int k = 0; k <= degree; ++k) coef[2 * k] = fc[k];

    // host copy of a device complex matrix [r][c]
    auto fetch = [&](int r, int c, std::vector<pvd::cd>& out) -> pv_status {
        std::vector<double> v((size_t)r * c * 2);
        PV_HIP(hipMemcpyAsync(v.data(), hd, v.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        PV_HIP(hipStreamSynchronize(s));
        out.resize((size_t)r * c);
        for (size_t i = 0; i < out.size(); ++i) {
            if (!std::isfinite(v[2 * i]) || !std::isfinite(v[2 * i + 1]))
                return fail(PV_ERR_NONFINITE, "Lanczos block holds non-finite values (start block or field)");
            out[i] = pvd::cd(v[2 * i], v[2 * i + 1]);
        }
        return PV_OK;
    };
    auto upload = [&](const std::vector<pvd::cd>& M) -> pv_status {
        std::vector<double> v(M.size() * 2);
        for (size_t i = 0; i < M.size(); ++i) {
            v[2 * i] = M[i].real();
            v[2 * i + 1] = M[i].imag();
        }
        PV_HIP(hipMemcpyAsync(hd, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, s));
        PV_HIP(hipStreamSynchronize(s));   // v goes out of scope
        return PV_OK;
    };
    // dst = src R^{-1} with src = Q R (Cholesky QR of nbl columns); R returned
    auto cholqr = [&](const void* src, void* dst, std::vector<pvd::cd>& R) -> pv_status {
        pv_status e = pv_gram(dtype, rows, nbl, nbl, src, src, hd, w + Lw.gp, gp_bytes, stream);
        if (e != PV_OK) return e;
        if ((e = fetch(nbl, nbl, R)) != PV_OK) return e;
        if (!pvd::cholesky_upper(nbl, R)) return fail(PV_ERR_NOT_CONVERGED, "Lanczos block lost rank");
        std::vector<pvd::cd> Ri;
        pvd::invert_upper(nbl, R, Ri);
        if ((e = upload(Ri)) != PV_OK) return e;
        return pv_block_rotate(dtype, rows, nbl, nbl, src, hd, 0, dst, stream);
    };
    auto matmul = [&](const std::vector<pvd::cd>& A, const std::vector<pvd::cd>& B2, int n) {
        std::vector<pvd::cd> C((size_t)n * n, pvd::cd(0, 0));
        for (int i = 0; i < n; ++i)
            for (int kk = 0; kk < n; ++kk)
                for (int j = 0; j < n; ++j) C[(size_t)i * n + j] += A[(size_t)i * n + kk] * B2[(size_t)kk * n + j];
        return C;
    };
    // orthonormal basis of src into S0 (two Cholesky QR passes); B = R2 R1
    auto orthonormalise = [&](const void* src, std::vector<pvd::cd>& B) -> pv_status {
        std::vector<pvd::cd> R1, R2;
        pv_status e = cholqr(src, T1, R1);
        if (e != PV_OK) return e;
        if ((e = cholqr(T1, S0, R2)) != PV_OK) return e;
        B = matmul(R2, R1, nbl);
        return PV_OK;
    };
    auto put_cols = [&](const void* src, int j0) -> pv_status {
        PV_HIP(pv::launch_column_copy(dtype, rows, nbl, src, nbl, 0, vblk(Lw.V, j0 / kTrBw), kTrBw, j0 % kTrBw,
                                      1.0, 0.0, s));
        return PV_OK;
    };

    PV_HIP(pv::launch_zero(w + Lw.V, Lw.vbw * Lw.nblk, s));
    std::vector<pvd::cd> B;
    if ((st = orthonormalise(v0, B)) != PV_OK) return st;
    if ((st = put_cols(S0, 0)) != PV_OK) return st;

    int k = 0, last = -1, it = 0;
    std::vector<double> kept, mu, th, rr;
    std::vector<pvd::cd> S, Y;      // restart couplings [nbl][k]; Ritz vectors of the projected matrix
    std::vector<int> keep;
    int nk = 0;
    bool converged = false;
    for (it = 1; it <= max_restarts; ++it) {
        std::vector<pvd::cd> T((size_t)m * m, pvd::cd(0, 0));
        for (int i = 0; i < k; ++i) T[(size_t)i * m + i] = kept[i];
        for (int r = 0; r < nbl; ++r)
            for (int i = 0; i < k; ++i) {
                T[(size_t)(k + r) * m + i] = S[(size_t)r * k + i];
                T[(size_t)i * m + k + r] = std::conj(S[(size_t)r * k + i]);
            }
        for (int j0 = k; j0 < m; j0 += nbl) {
            const int j1 = j0 + nbl;
            // Wv = p(H~) V_j   (V_j is in S0)
            if ((st = run_series(l, dtype, nbl, a, b, degree, coef.data(), S0, Wv, Wv, w + Lw.S1, w + Lw.S2, s)) !=
                PV_OK)
                return st;
            // full reorthogonalisation against the basis columns < j1, twice;
            // the first pass yields the diagonal block A_j
            std::vector<pvd::cd> Aj((size_t)nbl * nbl);
            for (int pass = 0; pass < 2; ++pass)
                for (int bb = 0; bb * kTrBw < j1; ++bb) {
                    if ((st = pv_gram(dtype, rows, kTrBw, nbl, vblk(Lw.V, bb), Wv, hd, w + Lw.gp, gp_bytes,
                                      stream)) != PV_OK)
                        return st;
                    std::vector<pvd::cd> h;
                    if ((st = fetch(kTrBw, nbl, h)) != PV_OK) return st;
                    for (int r = 0; r < kTrBw; ++r) {
                        const int col = bb * kTrBw + r;
                        for (int c = 0; c < nbl; ++c) {
                            pvd::cd& v = h[(size_t)r * nbl + c];
                            if (col >= j1) v = 0.0;
                            else if (pass == 0 && col >= j0) Aj[(size_t)(col - j0) * nbl + c] = v;
                            v = -v;
                        }
                    }
                    if ((st = upload(h)) != PV_OK) return st;
                    if ((st = pv_block_rotate(dtype, rows, kTrBw, nbl, vblk(Lw.V, bb), hd, 1, Wv, stream)) != PV_OK)
                        return st;
                }
            for (int r = 0; r < nbl; ++r)
                for (int c = 0; c < nbl; ++c)
                    T[(size_t)(j0 + r) * m + j0 + c] = 0.5 * (Aj[(size_t)r * nbl + c] + std::conj(Aj[(size_t)c * nbl + r]));
            if ((st = orthonormalise(Wv, B)) != PV_OK) return st;
            if (j1 < m)
                for (int r = 0; r < nbl; ++r)
                    for (int c = 0; c < nbl; ++c) {
                        T[(size_t)(j1 + r) * m + j0 + c] = B[(size_t)r * nbl + c];
                        T[(size_t)(j0 + c) * m + j1 + r] = std::conj(B[(size_t)r * nbl + c]);
                    }
            if ((st = put_cols(S0, j1)) != PV_OK) return st;
        }
        // Ritz pairs of p(H~); keep those above the threshold, rounded up to
        // whole blocks with the next largest ones
        pvd::heev_jacobi(m, T, mu, Y);
        int nw = 0;
        for (int i = 0; i < m; ++i)
            if (mu[i] > tau) ++nw;
        nk = std::min((nw + nbl - 1) / nbl * nbl, m - nbl);
        keep.resize(nk);
        for (int i = 0; i < nk; ++i) keep[i] = m - nk + i;
        // U = V Y_keep
        const int ukb = (nk + kTrBw - 1) / kTrBw;
        for (int cb = 0; cb < ukb; ++cb)
            for (int bb = 0; bb * kTrBw < m; ++bb) {
                std::vector<pvd::cd> q((size_t)kTrBw * kTrBw, pvd::cd(0, 0));
                for (int r = 0; r < kTrBw; ++r)
                    for (int c = 0; c < kTrBw; ++c) {
                        const int row = bb * kTrBw + r, col = cb * kTrBw + c;
                        if (row < m && col < nk) q[(size_t)r * kTrBw + c] = Y[(size_t)row * m + keep[col]];
                    }
                if ((st = upload(q)) != PV_OK) return st;
                if ((st = pv_block_rotate(dtype, rows, kTrBw, kTrBw, vblk(Lw.V, bb), hd, bb > 0, vblk(Lw.U, cb),
                                          stream)) != PV_OK)
                    return st;
            }
        // Rayleigh quotients and residuals with respect to H
        th.assign(nk, 0.0);
        rr.assign(nk, 0.0);
        {
            const std::vector<double> one(kTrBw, 1.0), zero(kTrBw, 0.0);
            const size_t spb = pv_spmmv_workspace_size(l, dtype, kTrBw);
            for (int cb = 0; cb < ukb; ++cb) {
                if ((st = pv_spmmv(l, dtype, kTrBw, vblk(Lw.U, cb), nullptr, w + Lw.HU, one.data(), zero.data(),
                                   zero.data(), 0, nullptr, w + Lw.sp, spb, stream)) != PV_OK)
                    return st;
                if ((st = pv_gram(dtype, rows, kTrBw, kTrBw, vblk(Lw.U, cb), w + Lw.HU, hd, w + Lw.gp, gp_bytes,
                                  stream)) != PV_OK)
                    return st;
                std::vector<pvd::cd> g;
                if ((st = fetch(kTrBw, kTrBw, g)) != PV_OK) return st;
                std::vector<double> sh(kTrBw, 0.0);
                for (int c = 0; c < kTrBw && cb * kTrBw + c < nk; ++c)
                    sh[c] = th[cb * kTrBw + c] = g[(size_t)c * kTrBw + c].real();
                if ((st = pv_spmmv(l, dtype, kTrBw, vblk(Lw.U, cb), nullptr, w + Lw.HU, one.data(), sh.data(),
                                   zero.data(), PV_DOT_YY, Dd, w + Lw.sp, spb, stream)) != PV_OK)
                    return st;
                std::vector<double> d((size_t)kTrBw * 4);
                PV_HIP(hipMemcpyAsync(d.data(), Dd, d.size() * sizeof(double), hipMemcpyDeviceToHost, s));
                PV_HIP(hipStreamSynchronize(s));
                for (int c = 0; c < kTrBw && cb * kTrBw + c < nk; ++c)
                    rr[cb * kTrBw + c] = std::sqrt(std::max(d[c * 4 + 3], 0.0));
            }
        }
        bool all = nw > 0;
        for (int i = 0; i < nk; ++i)
            if (mu[keep[i]] > tau && !(rr[i] <= tol)) all = false;
        if (all && nw == last) {
            converged = true;
            break;
        }
        last = nw;
        if (it == max_restarts) break;
        // thick restart: V[:, :nk] = U, the next block (in S0) after it, and
        // the couplings B_last Y[last block rows, keep]
        for (int cb = 0; cb < ukb; ++cb)
            PV_HIP(hipMemcpyAsync(vblk(Lw.V, cb), vblk(Lw.U, cb), Lw.vbw, hipMemcpyDeviceToDevice, s));
        if ((st = put_cols(S0, nk)) != PV_OK) return st;
        kept.assign(nk, 0.0);
        S.assign((size_t)nbl * nk, pvd::cd(0, 0));
        for (int i = 0; i < nk; ++i) {
            kept[i] = mu[keep[i]];
            for (int r = 0; r < nbl; ++r)
                for (int c = 0; c < nbl; ++c)
                    S[(size_t)r * nk + i] += B[(size_t)r * nbl + c] * Y[(size_t)(m - nbl + c) * m + keep[i]];
        }
        k = nk;
    }
    if (it > max_restarts) it = max_restarts;
    // the pairs above the threshold with theta inside the window (eigenvalues
    // just outside can pass the threshold), ascending; Ritz vectors into X
    std::vector<int> order;
    for (int i = 0; i < nk; ++i)
        if (mu[keep[i]] > tau && th[i] >= lam_l && th[i] <= lam_r) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int i, int j) { return th[i] < th[j]; });
    const int nf = int(order.size());
    for (int i = 0; i < nf; ++i) {
        theta[i] = th[order[i]];
        res[i] = rr[order[i]];
    }
    if (n_out > 0) {
        PV_HIP(pv::launch_zero(X, vec_bytes(l, dtype, n_out), s));
        for (int i = 0; i < nf && i < n_out; ++i) {
            const int src = order[i];
            PV_HIP(pv::launch_column_copy(dtype, rows, 1, vblk(Lw.U, src / kTrBw), kTrBw, src % kTrBw, X, n_out, i,
                                          1.0, 0.0, s));
        }
    }
    PV_HIP(hipStreamSynchronize(s));
    *n_found = nf;
    *restarts = it;
    if (!converged)
        return fail(PV_ERR_NOT_CONVERGED, "%d Ritz pairs in the window, not all converged after %d restarts", nf, it);
    return PV_OK;
}

// ---------------------------------------------------------------------------
// Batched KPM over independent lattices, captured into a HIP graph
// ---------------------------------------------------------------------------
struct pv_batch {
    std::vector<pv_lattice*> lats;
    int family = 0, n_orb = 0;
    // launch shape per (dtype, log2 nb) from pv_batch_autotune (kernel,
    // elems_per_lane, workgroup_size); unset: lattice 0's kernel and elements
    // per lane with 256-lane workgroups
    pv_tuning tune[2][7] = {};
    bool tuned[2][7] = {};
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> key;
    int captures = 0, replays = 0;
};

namespace {

// Chebyshev steps of each timed run of pv_batch_autotune
constexpr int kBatchTuneSteps = 8;

struct BatchLayout {
    size_t tables, block_inst, inst_block0, invD, partials, partial_stride, moments, vecs, total;
    std::vector<size_t> vec_off;  // per instance: A at vec_off[i], B at vec_off[i] + vb_i
    std::vector<int> nblocks;
    int total_blocks;
    int staged;
};

// Launch shape of a batch: its own (pv_batch_autotune) or, unset, lattice
// 0's kernel choice and elements per lane with 256-lane workgroups.
pv_tuning batch_shape(const pv_batch* B, int dtype, int nb) {
    const int di = dtype == PV_C128 ? 0 : 1, ni = log2_nb(nb);
    if (B->tuned[di][ni]) return B->tune[di][ni];
    pv_tuning t{};
    t.kernel = B->lats[0]->tune[di][ni].kernel;
    t.elems_per_lane = B->lats[0]->tune[di][ni].elems_per_lane;
    return t;
}

// A batch of generic-stencil lattices takes generated kernels when every
// instance would (set_codegen) and all share one pattern.
bool batch_codegen(const pv_batch* B) {
    if (B->family != pv::FAM_GENERIC) return false;
    for (const pv_lattice* l : B->lats)
        if (!uses_codegen(l) || l->cg_src != B->lats[0]->cg_src) return false;
    return true;
}

// Launch description of instance i of a batch (every instance takes the
// batch's shape).
pv::SweepParams batch_params(const pv_batch* B, int i, int dtype, int nb) {
    pv::SweepParams p = base_params(B->lats[i], dtype, nb);
    if (!batch_codegen(B)) p.cg_src = nullptr;
    p.vtype = (dtype == PV_C128) ? 0 : B->lats[i]->vtype;
    const pv_tuning t = batch_shape(B, dtype, nb);
    p.kernel = t.kernel;
    p.st_E = t.elems_per_lane;
    p.st_nt = t.workgroup_size;
    return p;
}

// The staged kernel serves a batch unless its shape asks for the direct one;
// by default only batches of instances averaging at least 2^20 elements per
// block (smaller ones are launch-latency bound).
bool batch_may_stage(const pv_batch* B, int dtype, int nb) {
    static const char* env = std::getenv("PV_SWEEP");
    if ((B->family == pv::FAM_GENERIC && !batch_codegen(B)) || (env && std::atoi(env) == 1)) return false;
    if (B->n_orb * nb > pv::STAGED_MAX_SITE) return false;
    const int kind = batch_shape(B, dtype, nb).kernel;
    if (kind != 0 || (env && std::atoi(env) == 2)) return kind != 1;
    int64_t elems = 0;
    for (const pv_lattice* l : B->lats) elems += l->n_rows * nb;
    return elems / int64_t(B->lats.size()) >= (int64_t(1) << 20);
}

pv_status batch_counts(const pv_batch* B, int dtype, int nb, int staged, std::vector<int>& nblocks, int& total) {
    const int n = int(B->lats.size());
    nblocks.assign(n, 0);
    total = 0;
    std::vector<char> rec(pv::batch_record_bytes());
    for (int i = 0; i < n; ++i) {
        const pv::SweepParams p = batch_params(B, i, dtype, nb);
        if (pv::batch_fill_record(p, staged, rec.data(), &nblocks[i]) != hipSuccess)
            return fail(PV_ERR_UNSUPPORTED, "instance %d: unsupported field / vector type combination", i);
        total += nblocks[i];
    }
    return PV_OK;
}

// Workspace layout for the direct or the staged kernel; the regions are
// sized for the larger of the two, so the layout does not depend on which.
pv_status batch_layout(const pv_batch* B, int dtype, int nb, int M, int staged, BatchLayout& L) {
    const int n = int(B->lats.size());
    pv_status st;
    std::vector<int> nd, ns;
    int td = 0, ts = 0;
    if ((st = batch_counts(B, dtype, nb, 0, nd, td)) != PV_OK) return st;
    const bool may = batch_may_stage(B, dtype, nb);
    if (may && (st = batch_counts(B, dtype, nb, 1, ns, ts)) != PV_OK) return st;
    L.staged = staged && may;
    L.nblocks = L.staged ? ns : nd;
    L.total_blocks = L.staged ? ts : td;
    const int cap = std::max(td, ts);
    size_t off = 0;
    L.tables = off; off += align_up(4 * (size_t)n * pv::batch_record_bytes());
    L.block_inst = off; off += align_up(sizeof(int) * cap);
    L.inst_block0 = off; off += align_up(sizeof(int) * (n + 1));
    L.invD = off; off += align_up(sizeof(double) * n);
    // two partial buffers: step n writes buffer n % 2 while its sweep folds
    // in the reduction of step n - 1 from the other
    L.partials = off; off += 2 * align_up((size_t)cap * nb * 4 * sizeof(double));
    L.partial_stride = align_up((size_t)cap * nb * 4 * sizeof(double));
    L.moments = off; off += align_up((size_t)n * nb * M * sizeof(double));
    L.vecs = off;
    L.vec_off.resize(n);
    for (int i = 0; i < n; ++i) {
        L.vec_off[i] = off;
        off += 2 * vec_bytes(B->lats[i], dtype, nb);
    }
    L.total = off;
    return PV_OK;
}

void release_graph(pv_batch* B) {
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
    B->key.clear();
}

}  // namespace

extern "C" pv_status pv_batch_create(int n, pv_lattice* const* lats, pv_batch** out) {
    if (!out || n < 1 || !lats) return fail(PV_ERR_INVALID_ARG, "pv_batch_create: need n >= 1 lattices");
    *out = nullptr;
    for (int i = 0; i < n; ++i)
        if (!lats[i]) return fail(PV_ERR_INVALID_ARG, "lattice %d is NULL", i);
    for (int i = 1; i < n; ++i)
        if (lats[i]->family != lats[0]->family || lats[i]->n_orb != lats[0]->n_orb)
            return fail(PV_ERR_UNSUPPORTED, "lattice %d has another stencil family than lattice 0", i);
    pv_batch* B = new (std::nothrow) pv_batch();
    if (!B) return fail(PV_ERR_OOM, "host allocation failed");
    B->lats.assign(lats, lats + n);
    B->family = lats[0]->family;
    B->n_orb = lats[0]->n_orb;
    *out = B;
    return PV_OK;
}

extern "C" void pv_batch_destroy(pv_batch* B) {
    if (!B) return;
    release_graph(B);
    if (B->cap) (void)hipStreamDestroy(B->cap);
    delete B;
}

extern "C" pv_status pv_batch_stats(const pv_batch* B, int* captures, int* replays) {
    if (!B) return fail(PV_ERR_INVALID_ARG, "batch is NULL");
    if (captures) *captures = B->captures;
    if (replays) *replays = B->replays;
    return PV_OK;
}

extern "C" size_t pv_batch_kpm_workspace_size(const pv_batch* B, int dtype, int nb, int M) {
    if (!B || !is_pow2(nb) || nb > PV_MAX_NB || (dtype != PV_C128 && dtype != PV_C64) || M < 2 || M > 65536) return 0;
    BatchLayout L;
    if (batch_layout(B, dtype, nb, M, 0, L) != PV_OK) return 0;
    return L.total;
}

extern "C" pv_status pv_batch_kpm_moments(pv_batch* B, int dtype, int nb, int M, const double* a, const double* b,
                                          const void* const* r, double* mu, void* work, size_t work_bytes,
                                          void* stream) {
    if (!B) return fail(PV_ERR_INVALID_ARG, "batch is NULL");
    pv_status st;
    const int n = int(B->lats.size());
    if ((st = check_nb(nb)) != PV_OK) return st;
    if (M < 2 || (M & 1) || M > 65536) return fail(PV_ERR_INVALID_ARG, "M = %d must be even, 2..65536", M);
    if (!a || !b || !r || !mu) return fail(PV_ERR_INVALID_ARG, "a, b, r and mu are required");
    for (int i = 0; i < n; ++i) {
        if ((st = check_dtype(B->lats[i], dtype)) != PV_OK) return st;
        if ((st = check_vec(r[i], dtype, "r[i]")) != PV_OK) return st;
        if (!(a[i] > 0.0) || !std::isfinite(a[i]) || !std::isfinite(b[i]))
            return fail(PV_ERR_INVALID_ARG, "instance %d: need finite a > 0 and b", i);
    }
    // the staged kernel reads the start blocks in 16-byte chunks
    int aligned = 1;
    for (int i = 0; i < n; ++i)
        if (reinterpret_cast<uintptr_t>(r[i]) % 16) aligned = 0;
    BatchLayout L;
    if ((st = batch_layout(B, dtype, nb, M, aligned, L)) != PV_OK) return st;
    if (!work || work_bytes < L.total) return fail(PV_ERR_WORKSPACE, "workspace %zu < %zu bytes", work_bytes, L.total);
    for (int i = 0; i < n; ++i)
        if ((st = ensure_device(B->lats[i])) != PV_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);

    // fingerprint of everything the captured graph bakes in; the graph writes
    // the moments into the workspace, so the caller's mu may move between calls
    const pv_tuning t0 = batch_shape(B, dtype, nb);
    std::vector<uint64_t> key = {(uint64_t)dtype, (uint64_t)nb, (uint64_t)M, (uint64_t)(uintptr_t)work,
                                 (uint64_t)work_bytes, (uint64_t)L.staged, (uint64_t)t0.kernel,
                                 (uint64_t)t0.elems_per_lane, (uint64_t)t0.workgroup_size,
                                 (uint64_t)batch_codegen(B)};
    char* const mu_ws = static_cast<char*>(work) + L.moments;
    const size_t mu_bytes = (size_t)n * nb * M * sizeof(double);
    for (int i = 0; i < n; ++i) {
        uint64_t ab[2];
        std::memcpy(&ab[0], &a[i], 8);
        std::memcpy(&ab[1], &b[i], 8);
        uint64_t rw;
        std::memcpy(&rw, &B->lats[i]->rng_W, 8);
        key.insert(key.end(), {(uint64_t)(uintptr_t)r[i], ab[0], ab[1], (uint64_t)(uintptr_t)B->lats[i]->V,
                               (uint64_t)B->lats[i]->vtype, (uint64_t)(uintptr_t)B->lats[i]->d_coef,
                               (uint64_t)B->lats[i]->rng_on, B->lats[i]->rng_seed, rw});
    }
    if (B->exec && key == B->key) {
        PV_HIP(hipGraphLaunch(B->exec, s));
        PV_HIP(hipMemcpyAsync(mu, mu_ws, mu_bytes, hipMemcpyDeviceToDevice, s));
        ++B->replays;
        return PV_OK;
    }
    release_graph(B);
    // a replay of the previous graph may still read the tables in `work`
    PV_HIP(hipStreamSynchronize(s));

    char* w = static_cast<char*>(work);
    const size_t rb = pv::batch_record_bytes();
    std::vector<char> tables(4 * (size_t)n * rb);
    std::vector<int> block_inst(L.total_blocks), inst_block0(n + 1);
    std::vector<double> invD(n);
    int b0 = 0;
    for (int i = 0; i < n; ++i) {
        pv_lattice* l = B->lats[i];
        inst_block0[i] = b0;
        for (int k = 0; k < L.nblocks[i]; ++k) block_inst[b0 + k] = i;
        b0 += L.nblocks[i];
        invD[i] = 1.0 / double(l->n_rows);
        void* A = w + L.vec_off[i];
        void* Bv = w + L.vec_off[i] + vec_bytes(l, dtype, nb);
        for (int v = 0; v < 4; ++v) {
            pv::SweepParams p = batch_params(B, i, dtype, nb);
            p.zero_row = l->d_zero;
            p.slab_rows = slab_rows(l, dtype, nb);
            // variants 0 and 2 run even steps, 1 and 3 odd ones: dots into
            // buffer v % 2; every step after the first folds in the previous
            // step's reduction (this instance's rows of the other buffer)
            double* part[2] = {reinterpret_cast<double*>(w + L.partials),
                               reinterpret_cast<double*>(w + L.partials + L.partial_stride)};
            p.partials = part[v & 1];
            if (v > 0) {
                p.red_src = part[(v & 1) ^ 1] + (size_t)inst_block0[i] * nb * 4;
                p.red_out = reinterpret_cast<double*>(mu_ws) + (size_t)i * nb * M;
                p.red_grid = L.nblocks[i];
                p.red_mode = v == 1 ? 1 : 2;
                p.red_M = M;
                p.red_invD = invD[i];
            }
            p.ep = pv::EP_STORE_Y | pv::EP_DOTS;
            p.beta = b[i];
            if (v == 0) {          // w_1 = H~ w_0
                p.x = r[i]; p.y = A; p.z = nullptr; p.alpha = 1.0 / a[i]; p.gamma = 0.0;
            } else if (v == 1) {   // w_2 = 2 H~ w_1 - w_0
                p.x = A; p.z = r[i]; p.y = Bv; p.alpha = 2.0 / a[i]; p.gamma = -1.0;
            } else if (v == 2) {   // even step n >= 2: x = B, in place over A
                p.x = Bv; p.z = A; p.y = A; p.alpha = 2.0 / a[i]; p.gamma = -1.0;
            } else {               // odd step n >= 3: x = A, in place over B
                p.x = A; p.z = Bv; p.y = Bv; p.alpha = 2.0 / a[i]; p.gamma = -1.0;
            }
            int nblk = 0;
            if (pv::batch_fill_record(p, L.staged, tables.data() + ((size_t)v * n + i) * rb, &nblk) != hipSuccess ||
                nblk != L.nblocks[i])
                return fail(PV_ERR_UNSUPPORTED, "instance %d: unsupported type combination", i);
        }
    }
    inst_block0[n] = b0;
    PV_HIP(hipMemcpy(w + L.tables, tables.data(), tables.size(), hipMemcpyHostToDevice));
    PV_HIP(hipMemcpy(w + L.block_inst, block_inst.data(), sizeof(int) * block_inst.size(), hipMemcpyHostToDevice));
    PV_HIP(hipMemcpy(w + L.inst_block0, inst_block0.data(), sizeof(int) * inst_block0.size(), hipMemcpyHostToDevice));
    PV_HIP(hipMemcpy(w + L.invD, invD.data(), sizeof(double) * n, hipMemcpyHostToDevice));

    if (!B->cap) PV_HIP(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
    const int* d_bi = reinterpret_cast<const int*>(w + L.block_inst);
    const int* d_i0 = reinterpret_cast<const int*>(w + L.inst_block0);
    const double* d_invD = reinterpret_cast<const double*>(w + L.invD);
    const double* d_part[2] = {reinterpret_cast<const double*>(w + L.partials),
                               reinterpret_cast<const double*>(w + L.partials + L.partial_stride)};
    const int vtype = (dtype == PV_C128) ? 0 : B->lats[0]->vtype;
    for (int i = 1; i < n; ++i)
        if (dtype != PV_C128 && B->lats[i]->vtype != vtype && (B->lats[i]->V || B->lats[0]->V))
            return fail(PV_ERR_UNSUPPORTED, "all instances of a batch need the same field type");
    pv::SweepParams p0 = batch_params(B, 0, dtype, nb);
    p0.vtype = vtype;
    p0.ep = pv::EP_STORE_Y | pv::EP_DOTS;
    // a generated kernel is compiled and loaded before the capture
    if (p0.cg_src) PV_HIP(pv::codegen_prepare_batch(p0, L.staged));
    PV_HIP(hipStreamBeginCapture(B->cap, hipStreamCaptureModeRelaxed));
    hipError_t e = hipSuccess;
    // one launch per step (each folds in the previous step's moments), then
    // the last step's reduction
    for (int step = 0; step < M / 2 && e == hipSuccess; ++step) {
        const int v = step == 0 ? 0 : (step == 1 ? 1 : (step % 2 == 0 ? 2 : 3));
        e = pv::launch_batch_sweep(p0, L.staged, w + L.tables + (size_t)v * n * rb, d_bi, d_i0, L.total_blocks,
                                   step - 1, B->cap);
    }
    const int last = M / 2 - 1;
    if (e == hipSuccess)
        e = pv::launch_batch_reduce(d_part[last & 1], d_i0, n, nb, last == 0 ? 1 : 2,
                                    reinterpret_cast<double*>(mu_ws), M, last, d_invD, B->cap);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(B->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(e != hipSuccess ? e : e2, "batched KPM graph capture");
    }
    B->graph = g;
    PV_HIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    B->key = key;
    ++B->captures;
    PV_HIP(hipGraphLaunch(B->exec, s));
    PV_HIP(hipMemcpyAsync(mu, mu_ws, mu_bytes, hipMemcpyDeviceToDevice, s));
    return PV_OK;
}

extern "C" pv_status pv_batch_set_tuning(pv_batch* B, int dtype, int nb, const pv_tuning* t) {
    if (!B) return fail(PV_ERR_INVALID_ARG, "batch is NULL");
    pv_status st;
    if (dtype != PV_C128 && dtype != PV_C64) return fail(PV_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    if ((st = check_nb(nb)) != PV_OK) return st;
    if (t && (st = check_tuning(dtype, *t)) != PV_OK) return st;
    if (t && t->workgroup_size == 512 && B->family == pv::FAM_GENERIC && !batch_codegen(B))
        return fail(PV_ERR_UNSUPPORTED,
                    "512-lane batched sweeps need a compiled stencil family or generated kernels of one pattern");
    const int di = dtype == PV_C128 ? 0 : 1, ni = log2_nb(nb);
    pv_tuning z{};
    if (t) {
        // a batch takes the kernel, elements per lane and lanes per
        // workgroup; every instance walks whole columns
        z.kernel = t->kernel;
        z.elems_per_lane = t->elems_per_lane;
        z.workgroup_size = t->workgroup_size;
    }
    B->tune[di][ni] = z;
    B->tuned[di][ni] = t != nullptr;
    release_graph(B);
    return PV_OK;
}

extern "C" pv_status pv_batch_get_tuning(const pv_batch* B, int dtype, int nb, pv_tuning* t) {
    if (!B || !t) return fail(PV_ERR_INVALID_ARG, "batch or output is NULL");
    pv_status st;
    if (dtype != PV_C128 && dtype != PV_C64) return fail(PV_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    if ((st = check_nb(nb)) != PV_OK) return st;
    *t = batch_shape(B, dtype, nb);
    return PV_OK;
}

namespace {

// Launch shapes pv_batch_autotune times: the direct kernel; the staged one
// with each elements per lane and 256 or 512 lanes
std::vector<pv_tuning> batch_tune_candidates(const pv_batch* B, int dtype, int nb) {
    std::vector<pv_tuning> cand;
    pv_tuning t{};
    t.kernel = 1;
    cand.push_back(t);
    if ((B->family != pv::FAM_GENERIC || batch_codegen(B)) && B->n_orb * nb <= pv::STAGED_MAX_SITE)
        for (int wg : {0, 512})
            for (int e : {dtype == PV_C128 ? 1 : 2, dtype == PV_C128 ? 2 : 4}) {
                t = pv_tuning{};
                t.kernel = 2;
                t.elems_per_lane = e;
                t.workgroup_size = wg;
                cand.push_back(t);
            }
    return cand;
}

// Workspace of the timed runs: the block counts, hence the layout, depend on
// the launch shape, so the largest over the candidates (0: unsupported)
size_t batch_tune_kpm_bytes(const pv_batch* B, int dtype, int nb) {
    pv_batch probe;   // the batch's lattices under one candidate shape (no graph)
    probe.lats = B->lats;
    probe.family = B->family;
    probe.n_orb = B->n_orb;
    const int di = dtype == PV_C128 ? 0 : 1, ni = log2_nb(nb);
    size_t most = 0;
    for (const pv_tuning& t : batch_tune_candidates(B, dtype, nb)) {
        probe.tune[di][ni] = t;
        probe.tuned[di][ni] = true;
        const size_t k = pv_batch_kpm_workspace_size(&probe, dtype, nb, 2 * kBatchTuneSteps);
        if (!k) return 0;
        most = std::max(most, k);
    }
    return most;
}

}  // namespace

extern "C" size_t pv_batch_autotune_workspace_size(const pv_batch* B, int dtype, int nb) {
    if (!B || !is_pow2(nb) || nb > PV_MAX_NB || (dtype != PV_C128 && dtype != PV_C64)) return 0;
    const size_t kpm = batch_tune_kpm_bytes(B, dtype, nb);
    if (!kpm) return 0;
    return kpm + align_up(B->lats.size() * (size_t)nb * 2 * kBatchTuneSteps * sizeof(double));
}

extern "C" pv_status pv_batch_autotune(pv_batch* B, int dtype, int nb, const double* a, const double* b,
                                       const void* const* r, void* work, size_t work_bytes, void* stream,
                                       pv_tuning* out, double* ms_out) {
    if (!B) return fail(PV_ERR_INVALID_ARG, "batch is NULL");
    pv_status st;
    if ((st = check_nb(nb)) != PV_OK) return st;
    if (dtype != PV_C128 && dtype != PV_C64) return fail(PV_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    const int M = 2 * kBatchTuneSteps;
    const size_t need_kpm = batch_tune_kpm_bytes(B, dtype, nb);
    const size_t need = pv_batch_autotune_workspace_size(B, dtype, nb);
    if (!need) return fail(PV_ERR_INVALID_ARG, "batch does not take dtype %d with nb = %d", dtype, nb);
    if (!work || work_bytes < need) return fail(PV_ERR_WORKSPACE, "workspace %zu < %zu bytes", work_bytes, need);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int di = dtype == PV_C128 ? 0 : 1, ni = log2_nb(nb);
    const pv_tuning saved = B->tune[di][ni];
    const bool saved_set = B->tuned[di][ni];
    // moments of the timed runs, after the runs' own workspace
    double* mu = reinterpret_cast<double*>(static_cast<char*>(work) + need_kpm);
    hipEvent_t e0, e1;
    PV_HIP(hipEventCreate(&e0));
    PV_HIP(hipEventCreate(&e1));
    // time of one step of the captured batch under shape t: the first call
    // captures, then the fastest of three replays of kBatchTuneSteps steps
    auto measure = [&](const pv_tuning& t, double& ms) -> pv_status {
        B->tune[di][ni] = t;
        B->tuned[di][ni] = true;
        pv_status e = pv_batch_kpm_moments(B, dtype, nb, M, a, b, r, mu, work, need_kpm, stream);
        if (e != PV_OK) return e;
        ms = 1e300;
        for (int k = 0; k < 3; ++k) {
            PV_HIP(hipEventRecord(e0, s));
            if ((e = pv_batch_kpm_moments(B, dtype, nb, M, a, b, r, mu, work, need_kpm, stream)) != PV_OK) return e;
            PV_HIP(hipEventRecord(e1, s));
            PV_HIP(hipEventSynchronize(e1));
            float tt = 0.f;
            PV_HIP(hipEventElapsedTime(&tt, e0, e1));
            ms = std::min(ms, double(tt) / kBatchTuneSteps);
        }
        return PV_OK;
    };
    const std::vector<pv_tuning> cand = batch_tune_candidates(B, dtype, nb);
    pv_tuning best{};
    double best_ms = 1e300;
    pv_status err = PV_OK;
    for (const pv_tuning& t : cand) {
        double ms = 0.0;
        if ((err = measure(t, ms)) != PV_OK) break;
        if (ms < 0.99 * best_ms) {
            best_ms = ms;
            best = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != PV_OK) {
        B->tune[di][ni] = saved;
        B->tuned[di][ni] = saved_set;
        release_graph(B);
        return err;
    }
    B->tune[di][ni] = best;
    B->tuned[di][ni] = true;
    release_graph(B);
    if (out) *out = best;
    if (ms_out) *ms_out = best_ms;
    return PV_OK;
}

// ---------------------------------------------------------------------------
// Adjoints with respect to the on-site field (gradients of KPM moments and
// of Chebyshev propagation)
// ---------------------------------------------------------------------------
namespace {

pv_status check_grad_args(pv_lattice* l, int dtype, int nb, double a, double b, const double* gradV) {
    pv_status st;
    if ((st = check_series_args(l, dtype, nb, a, b)) != PV_OK) return st;
    if (l->pot_mode == PV_POT_NONE) return fail(PV_ERR_INVALID_ARG, "lattice has no on-site field to differentiate");
    if (l->pot_mode == PV_POT_SITE && l->n_orb * nb > 64)
        return fail(PV_ERR_UNSUPPORTED, "gradient of a site field needs n_orb * nb <= 64");
    if (!gradV) return fail(PV_ERR_INVALID_ARG, "gradV is NULL");
    return PV_OK;
}

size_t grad_len(const pv_lattice* l) { return size_t(l->pot_mode == PV_POT_ORBITAL ? l->n_rows : l->n_sites); }

// One sweep y = alpha (H - beta) x + gamma z with the adjoint epilogue.
pv_status adjoint_sweep(pv_lattice* l, int dtype, int nb, const void* x, const void* z, void* y, double alpha,
                        double beta, double gamma, const void* w0, const void* w1, const void* w2,
                        const double* gcoef, double* grad, double gx, double gy, unsigned ep, hipStream_t s) {
    pv::SweepParams p = base_params(l, dtype, nb);
    pv_status st;
    if ((st = fill_traversal(l, dtype, nb, p)) != PV_OK) return st;
    p.x = x;
    p.z = z;
    p.y = y;
    p.alpha = alpha;
    p.beta = beta;
    p.gamma = gamma;
    p.gw[0] = w0;
    p.gw[1] = w1;
    p.gw[2] = w2;
    p.gcoef = gcoef;
    p.grad = grad;
    p.gx = gx;
    p.gy = gy;
    p.grad_mode = l->pot_mode;
    p.ep = ep;
    PV_HIP(pv::launch_sweep(p, num_cus(), s));
    return PV_OK;
}

}  // namespace

namespace {
// KPM adjoint workspace: 2J checkpoint vectors (w_{jC}, w_{jC+1}), C segment
// vectors, two adjoint and two forward vectors, the source-term table, then
// the dot partials of pv_kpm_moments_ckpt.
// Intervals beyond N = M/2 all mean one segment; the layout takes C = min(ckpt, N).
size_t kpm_vjp_core_bytes(const pv_lattice* l, int dtype, int nb, int M, int ckpt) {
    const int N = M / 2, C = std::min(ckpt, N), J = (N - 1) / C + 1;
    const size_t vb = vec_bytes(l, dtype, nb);
    return vb * (2 * (size_t)J + C + 2 + 2) + align_up((size_t)(N + 1) * 3 * nb * 2 * sizeof(double));
}
}  // namespace

extern "C" size_t pv_kpm_vjp_workspace_size(const pv_lattice* l, int dtype, int nb, int M, int ckpt) {
    if (!l || !is_pow2(nb) || nb > PV_MAX_NB || M < 2 || (M & 1) || ckpt < 1 ||
        (dtype != PV_C128 && dtype != PV_C64))
        return 0;
    return kpm_vjp_core_bytes(l, dtype, nb, M, ckpt) + 2 * partial_bytes(l, nb);
}

namespace {

pv_status check_kpm_vjp_args(pv_lattice* l, int dtype, int nb, int M, double a, double b, const void* r,
                             const double* gbar, double* gradV, int ckpt, void* work, size_t work_bytes) {
    pv_status st;
    if (!l) return fail(PV_ERR_INVALID_ARG, "lattice is NULL");
    if ((st = check_grad_args(l, dtype, nb, a, b, gradV)) != PV_OK) return st;
    if ((st = check_vec(r, dtype, "r")) != PV_OK) return st;
    if (M < 2 || (M & 1) || M > 65536) return fail(PV_ERR_INVALID_ARG, "M = %d must be even, 2..65536", M);
    if (!gbar) return fail(PV_ERR_INVALID_ARG, "gbar is NULL");
    if (ckpt < 1) return fail(PV_ERR_INVALID_ARG, "checkpoint interval must be >= 1");
    const size_t need = pv_kpm_vjp_workspace_size(l, dtype, nb, M, ckpt);
    if (!work || work_bytes < need) return fail(PV_ERR_WORKSPACE, "workspace %zu < %zu bytes", work_bytes, need);
    return ensure_device(l);
}

// The adjoint sweep; with have_ckpt the checkpoint pairs are already in the
// workspace (pv_kpm_moments_ckpt) and the forward recurrence is skipped.
pv_status kpm_vjp_impl(pv_lattice* l, int dtype, int nb, int M, double a, double b, const void* r,
                       const double* gbar, double* gradV, int ckpt, void* work, hipStream_t s, bool have_ckpt) {
    pv_status st;
    const int N = M / 2, C = std::min(ckpt, N), J = (N - 1) / C + 1;
    const size_t vb = vec_bytes(l, dtype, nb);
    const double invD = 1.0 / double(l->n_rows);
    char* w = static_cast<char*>(work);
    auto ck = [&](int j, int which) { return static_cast<void*>(w + vb * (2 * (size_t)j + which)); };
    char* S = w + vb * 2 * (size_t)J;                  // C segment vectors
    void* L0 = S + vb * C;
    void* L1 = S + vb * (C + 1);
    void* F0 = S + vb * (C + 2);                       // forward ring
    void* F1 = S + vb * (C + 3);
    double* table = reinterpret_cast<double*>(S + vb * (C + 4));

    // cotangent of the moments -> coefficients of the adjoint source terms,
    // on the device (no host round trip)
    PV_HIP(pv::launch_kpm_adjoint_table(gbar, nb, M, invD, table, s));
    PV_HIP(pv::launch_zero(gradV, grad_len(l) * sizeof(double), s));
    PV_HIP(pv::launch_zero(L0, vb, s));
    PV_HIP(pv::launch_zero(L1, vb, s));
    const size_t vbytes = (size_t)l->n_rows * nb * elem_bytes(dtype);

    // forward recurrence, keeping (w_{jC}, w_{jC+1}) for j = 0..J-1
    const unsigned store = pv::EP_STORE_Y;
    if (!have_ckpt) {
        if ((st = adjoint_sweep(l, dtype, nb, r, nullptr, F0, 1.0 / a, b, 0.0, nullptr, nullptr, nullptr, nullptr,
                                nullptr, 0, 0, store, s)) != PV_OK)
            return st;
        PV_HIP(pv::launch_copy(r, ck(0, 0), vbytes, s));
        PV_HIP(pv::launch_copy(F0, ck(0, 1), vbytes, s));
        {
            const void* prev = r;
            void* cur = F0;
            for (int k = 1; k <= (J - 1) * C; ++k) {
                void* next = (k == 1) ? F1 : const_cast<void*>(prev);
                if ((st = adjoint_sweep(l, dtype, nb, cur, prev, next, 2.0 / a, b, -1.0, nullptr, nullptr, nullptr,
                                        nullptr, nullptr, 0, 0, store, s)) != PV_OK)
                    return st;
                prev = cur;
                cur = next;
                if (k % C == 0) {
                    PV_HIP(pv::launch_copy(prev, ck(k / C, 0), vbytes, s));
                    PV_HIP(pv::launch_copy(cur, ck(k / C, 1), vbytes, s));
                }
            }
        }
    }

    // reverse sweep over segments: recompute w_{jC}..w_{min((j+1)C+1, N)}, then
    // lambda_k = G_k + 2 H~ lambda_{k+1} - lambda_{k+2} for k = min((j+1)C, N)..jC+1
    void* lx = L0;   // lambda_{k+1}
    void* lz = L1;   // lambda_{k+2}, overwritten by lambda_k
    for (int j = J - 1; j >= 0; --j) {
        const int k_hi = std::min((j + 1) * C, N);
        // w_{(j+1)C} and w_{(j+1)C+1} are the next segment's checkpoint pair
        auto wv = [&](int i) -> void* {
            if (i == j * C) return ck(j, 0);
            if (i == j * C + 1) return ck(j, 1);
            if (j + 1 < J && i == (j + 1) * C) return ck(j + 1, 0);
            if (j + 1 < J && i == (j + 1) * C + 1) return ck(j + 1, 1);
            return S + vb * (size_t)(i - j * C - 2);
        };
        // recompute the rest (with one segment, pv_kpm_moments_ckpt left
        // w_2..w_N in place)
        const bool stored = have_ckpt && J == 1;
        const int i_hi = (j + 1 < J) ? (j + 1) * C - 1 : std::min(k_hi + 1, N);
        for (int i = j * C + 2; !stored && i <= i_hi; ++i)
            if ((st = adjoint_sweep(l, dtype, nb, wv(i - 1), wv(i - 2), wv(i), 2.0 / a, b, -1.0, nullptr, nullptr,
                                    nullptr, nullptr, nullptr, 0, 0, store, s)) != PV_OK)
                return st;
        for (int k = k_hi; k >= j * C + 1; --k) {
            if ((st = adjoint_sweep(l, dtype, nb, lx, lz, lz, 2.0 / a, b, -1.0, wv(k - 1), wv(k),
                                    k < N ? wv(k + 1) : nullptr, table + (size_t)k * 3 * nb * 2, gradV, 2.0 / a,
                                    k == 1 ? 1.0 / a : 0.0, store | pv::EP_GTERMS | pv::EP_GRAD, s)) != PV_OK)
                return st;
            std::swap(lx, lz);
        }
    }
    return PV_OK;
}

}  // namespace

extern "C" pv_status pv_kpm_moments_vjp(pv_lattice* l, int dtype, int nb, int M, double a, double b, const void* r,
                                        const double* gbar, double* gradV, int ckpt, void* work, size_t work_bytes,
                                        void* stream) {
    pv_status st;
    if ((st = check_kpm_vjp_args(l, dtype, nb, M, a, b, r, gbar, gradV, ckpt, work, work_bytes)) != PV_OK) return st;
    return kpm_vjp_impl(l, dtype, nb, M, a, b, r, gbar, gradV, ckpt, work, static_cast<hipStream_t>(stream), false);
}

extern "C" pv_status pv_kpm_moments_ckpt(pv_lattice* l, int dtype, int nb, int M, double a, double b, const void* r,
                                         double* mu, int ckpt, void* work, size_t work_bytes, void* stream) {
    pv_status st;
    if ((st = check_kpm_args(l, dtype, nb, M, a, b, r, mu)) != PV_OK) return st;
    if (ckpt < 1) return fail(PV_ERR_INVALID_ARG, "checkpoint interval must be >= 1");
    const size_t need = pv_kpm_vjp_workspace_size(l, dtype, nb, M, ckpt);
    if (!work || work_bytes < need) return fail(PV_ERR_WORKSPACE, "workspace %zu < %zu bytes", work_bytes, need);
    if ((st = ensure_device(l)) != PV_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int N = M / 2, C = std::min(ckpt, N), J = (N - 1) / C + 1;
    const size_t vb = vec_bytes(l, dtype, nb);
    const size_t vbytes = (size_t)l->n_rows * nb * elem_bytes(dtype);
    char* w = static_cast<char*>(work);
    auto ck = [&](int j, int which) { return static_cast<void*>(w + vb * (2 * (size_t)j + which)); };
    char* S = w + vb * 2 * (size_t)J;
    void* F[2] = {S + vb * (C + 2), S + vb * (C + 3)};
    char* part = w + kpm_vjp_core_bytes(l, dtype, nb, M, ckpt);
    PV_HIP(pv::launch_copy(r, ck(0, 0), vbytes, s));
    // w_k goes straight to its checkpoint slot (jC + rem, rem in {0, 1});
    // with one segment (C >= M/2) w_2..w_N go to the segment slots, where
    // the adjoint reads them without recomputing; else to the forward ring
    // by parity.  With C = 1, w_k also fills slot (k - 1, 1).
    auto wbuf = [&](int k) -> void* {
        const int j = k / C, rem = k - j * C;
        if (j < J && rem <= 1) return ck(j, rem);
        if (J == 1 && k >= 2) return S + vb * (size_t)(k - 2);
        return F[k & 1];
    };
    auto after = [&](int k, const void* y) -> hipError_t {
        if (C == 1 && k - 1 < J) return pv::launch_copy(y, ck(k - 1, 1), vbytes, s);
        return hipSuccess;
    };
    return kpm_forward(l, dtype, nb, M, a, b, r, mu, reinterpret_cast<double*>(part),
                       reinterpret_cast<double*>(part + partial_bytes(l, nb)), wbuf, after, s);
}

extern "C" pv_status pv_kpm_moments_vjp_ckpt(pv_lattice* l, int dtype, int nb, int M, double a, double b,
                                             const void* r, const double* gbar, double* gradV, int ckpt, void* work,
                                             size_t work_bytes, void* stream) {
    pv_status st;
    if ((st = check_kpm_vjp_args(l, dtype, nb, M, a, b, r, gbar, gradV, ckpt, work, work_bytes)) != PV_OK) return st;
    return kpm_vjp_impl(l, dtype, nb, M, a, b, r, gbar, gradV, ckpt, work, static_cast<hipStream_t>(stream), true);
}

extern "C" size_t pv_cheb_propagate_vjp_workspace_size(const pv_lattice* l, int dtype, int nb, int M, int nsteps) {
    if (!l || !is_pow2(nb) || nb > PV_MAX_NB || M < 1 || nsteps < 1 || (dtype != PV_C128 && dtype != PV_C64))
        return 0;
    const size_t vb = vec_bytes(l, dtype, nb);
    return vb * ((size_t)nsteps + M + 4) + align_up((size_t)(M + 1) * 3 * nb * 2 * sizeof(double));
}

namespace {

// Series coefficients of one propagation step: eta_0 = e^{-ibdt} c_0,
// eta_k = 2 e^{-ibdt} c_k (complex interleaved, k = 0..M).
std::vector<double> tp_step_coefficients(double a, double b, double dt, int M) {
    std::vector<double> coef(2 * (M + 1));
    pv_cheb_tp_coefficients(a, dt, M, coef.data());
    const std::complex<double> ph = std::exp(std::complex<double>(0.0, -b * dt));
    for (int k = 0; k <= M; ++k) {
        std::complex<double> c(coef[2 * k], coef[2 * k + 1]);
        c *= ph * (k ? 2.0 : 1.0);
        coef[2 * k] = c.real();
        coef[2 * k + 1] = c.imag();
    }
    return coef;
}

// Workspace of the propagation adjoint: states psi_1..psi_{nsteps-1} in
// slots 1..nsteps-1, w_1..w_M, two adjoint and two cotangent vectors, the
// source-term table.
// With the series kept, w_k of step i (k = 1..M) follows at series(i, k).
struct TpVjpLayout {
    char* w;
    size_t vb;
    int nsteps, M;
    size_t base;   // bytes of the layout without the kept series
    void* state(int i) const { return w + vb * (size_t)i; }
    void* wk(int k) const { return w + vb * ((size_t)nsteps + k - 1); }
    void* L0() const { return w + vb * ((size_t)nsteps + M); }
    void* series(int i, int k) const { return w + base + vb * ((size_t)i * M + k - 1); }
};

// The forward of the adjoint: psi_{i+1} = U psi_i for i < n_keep, each kept
// in its state slot; with out != NULL the last step U psi_{nsteps-1} goes
// to out.
pv_status tp_forward_keep(pv_lattice* l, int dtype, int nb, double a, double b, int M, int nsteps, const double* coef,
                          const void* psi0, void* out, const TpVjpLayout& T, bool keep_series, hipStream_t s) {
    pv_status st;
    auto psi = [&](int i) -> const void* { return i == 0 ? psi0 : T.state(i); };
    for (int i = 0; i < nsteps; ++i) {
        void* dst = i + 1 < nsteps ? T.state(i + 1) : out;
        if (!dst) break;
        if (keep_series)
            st = run_series_keep(l, dtype, nb, a, b, M, coef, psi(i), dst, dst,
                                 [&](int k) { return T.series(i, k); }, s);
        else
            st = run_series(l, dtype, nb, a, b, M, coef, psi(i), dst, dst, T.wk(1), M >= 2 ? T.wk(2) : T.L0(), s);
        if (st != PV_OK) return st;
    }
    return PV_OK;
}

pv_status check_tp_vjp_args(pv_lattice* l, int dtype, int nb, double a, double b, double dt, int M, int nsteps,
                            const void* psi0, const void* psibar, void* psi0bar, double* gradV, void* work,
                            size_t work_bytes, int keep_series) {
    pv_status st;
    if (!l) return fail(PV_ERR_INVALID_ARG, "lattice is NULL");
    if ((st = check_grad_args(l, dtype, nb, a, b, gradV)) != PV_OK) return st;
    if ((st = check_vec(psi0, dtype, "psi0")) != PV_OK) return st;
    if ((st = check_vec(psibar, dtype, "psibar")) != PV_OK) return st;
    if (psi0bar && (st = check_vec(psi0bar, dtype, "psi0bar")) != PV_OK) return st;
    if (M < 1 || nsteps < 1 || !std::isfinite(dt)) return fail(PV_ERR_INVALID_ARG, "need M >= 1, nsteps >= 1");
    const size_t need = pv_cheb_propagate_keep_workspace_size(l, dtype, nb, M, nsteps, keep_series);
    if (!work || work_bytes < need) return fail(PV_ERR_WORKSPACE, "workspace %zu < %zu bytes", work_bytes, need);
    return ensure_device(l);
}

// The propagation adjoint; with have_states the states psi_1..psi_{nsteps-1}
// are already in the workspace (pv_cheb_propagate_keep).
pv_status tp_vjp_impl(pv_lattice* l, int dtype, int nb, double a, double b, double dt, int M, int nsteps,
                      const void* psi0, const void* psibar, void* psi0bar, double* gradV, void* work, hipStream_t s,
                      bool have_states, bool have_series) {
    pv_status st;
    const size_t vb = vec_bytes(l, dtype, nb);
    const size_t vbytes = (size_t)l->n_rows * nb * elem_bytes(dtype);
    char* w = static_cast<char*>(work);
    auto state = [&](int i) -> void* { return w + vb * (size_t)i; };          // psi_1 .. psi_{nsteps-1} (slot 0 unused)
    auto wk = [&](int k) -> void* { return w + vb * ((size_t)nsteps + k - 1); };  // w_1 .. w_M
    void* L0 = w + vb * ((size_t)nsteps + M);
    void* L1 = w + vb * ((size_t)nsteps + M + 1);
    void* Y0 = w + vb * ((size_t)nsteps + M + 2);
    void* Y1 = w + vb * ((size_t)nsteps + M + 3);
    double* table = reinterpret_cast<double*>(w + vb * ((size_t)nsteps + M + 4));

    const std::vector<double> coef = tp_step_coefficients(a, b, dt, M);
    // adjoint source of lambda_k: conj(eta_k) * Ybar in the third slot
    std::vector<double> tab((size_t)(M + 1) * 3 * nb * 2, 0.0);
    for (int k = 0; k <= M; ++k)
        for (int c = 0; c < nb; ++c) {
            double* row = &tab[(size_t)k * 3 * nb * 2];
            row[(2 * nb + c) * 2] = coef[2 * k];
            row[(2 * nb + c) * 2 + 1] = -coef[2 * k + 1];
        }
    PV_HIP(hipMemcpyAsync(table, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, s));
    PV_HIP(pv::launch_zero(gradV, grad_len(l) * sizeof(double), s));

    // forward: psi_{i+1} = U psi_i, keep psi_1 .. psi_{nsteps-1}
    auto psi = [&](int i) -> const void* { return i == 0 ? psi0 : state(i); };
    const TpVjpLayout T{w, vb, nsteps, M, pv_cheb_propagate_vjp_workspace_size(l, dtype, nb, M, nsteps)};
    if (!have_states &&
        (st = tp_forward_keep(l, dtype, nb, a, b, M, nsteps, coef.data(), psi0, nullptr, T, false, s)) != PV_OK)
        return st;

    PV_HIP(pv::launch_copy(psibar, Y0, vbytes, s));
    void* ybar = Y0;
    void* ynew = Y1;
    const unsigned store = pv::EP_STORE_Y;
    for (int i = nsteps - 1; i >= 0; --i) {
        const void* X = psi(i);
        // w_1 .. w_M of this step: kept by the forward, or recomputed
        auto wv = [&](int k) -> const void* { return k == 0 ? X : (have_series ? T.series(i, k) : wk(k)); };
        if (!have_series) {
            if ((st = adjoint_sweep(l, dtype, nb, X, nullptr, wk(1), 1.0 / a, b, 0.0, nullptr, nullptr, nullptr,
                                    nullptr, nullptr, 0, 0, store, s)) != PV_OK)
                return st;
            for (int k = 2; k <= M; ++k)
                if ((st = adjoint_sweep(l, dtype, nb, wv(k - 1), wv(k - 2), wk(k), 2.0 / a, b, -1.0, nullptr,
                                        nullptr, nullptr, nullptr, nullptr, 0, 0, store, s)) != PV_OK)
                    return st;
        }
        PV_HIP(pv::launch_zero(L0, vb, s));
        PV_HIP(pv::launch_zero(L1, vb, s));
        void* lx = L0;
        void* lz = L1;
        for (int k = M; k >= 1; --k) {
            if ((st = adjoint_sweep(l, dtype, nb, lx, lz, lz, 2.0 / a, b, -1.0, wv(k - 1), wv(k), ybar,
                                    table + (size_t)k * 3 * nb * 2, gradV, 2.0 / a, k == 1 ? 1.0 / a : 0.0,
                                    store | pv::EP_GTERMS | pv::EP_GRAD, s)) != PV_OK)
                return st;
            std::swap(lx, lz);
        }
        // lambda_0 = conj(eta_0) Ybar + H~ lambda_1 - lambda_2  ->  cotangent of psi_i
        if ((st = adjoint_sweep(l, dtype, nb, lx, lz, ynew, 1.0 / a, b, -1.0, nullptr, nullptr, ybar, table, nullptr,
                                0, 0, store | pv::EP_GTERMS, s)) != PV_OK)
            return st;
        std::swap(ybar, ynew);
    }
    if (psi0bar) PV_HIP(pv::launch_copy(ybar, psi0bar, vbytes, s));
    return PV_OK;
}

}  // namespace

extern "C" pv_status pv_cheb_propagate_vjp(pv_lattice* l, int dtype, int nb, double a, double b, double dt, int M,
                                           int nsteps, const void* psi0, const void* psibar, void* psi0bar,
                                           double* gradV, void* work, size_t work_bytes, void* stream) {
    pv_status st;
    if ((st = check_tp_vjp_args(l, dtype, nb, a, b, dt, M, nsteps, psi0, psibar, psi0bar, gradV, work, work_bytes,
                                0)) != PV_OK)
        return st;
    return tp_vjp_impl(l, dtype, nb, a, b, dt, M, nsteps, psi0, psibar, psi0bar, gradV, work,
                       static_cast<hipStream_t>(stream), false, false);
}

extern "C" size_t pv_cheb_propagate_keep_workspace_size(const pv_lattice* l, int dtype, int nb, int M, int nsteps,
                                                        int keep_series) {
    const size_t base = pv_cheb_propagate_vjp_workspace_size(l, dtype, nb, M, nsteps);
    if (base == 0 || !keep_series) return base;
    return base + vec_bytes(l, dtype, nb) * (size_t)nsteps * (size_t)M;
}

extern "C" pv_status pv_cheb_propagate_keep(pv_lattice* l, int dtype, int nb, double a, double b, double dt, int M,
                                            int nsteps, const void* psi0, void* psiT, int keep_series, void* work,
                                            size_t work_bytes, void* stream) {
    pv_status st;
    if ((st = check_series_args(l, dtype, nb, a, b)) != PV_OK) return st;
    if ((st = check_vec(psi0, dtype, "psi0")) != PV_OK) return st;
    if ((st = check_vec(psiT, dtype, "psiT")) != PV_OK) return st;
    if (psiT == psi0) return fail(PV_ERR_INVALID_ARG, "psiT must not alias psi0 (the adjoint reads psi0)");
    if (M < 1 || nsteps < 1 || !std::isfinite(dt)) return fail(PV_ERR_INVALID_ARG, "need M >= 1, nsteps >= 1");
    const size_t need = pv_cheb_propagate_keep_workspace_size(l, dtype, nb, M, nsteps, keep_series);
    if (!work || work_bytes < need) return fail(PV_ERR_WORKSPACE, "workspace %zu < %zu bytes", work_bytes, need);
    if ((st = ensure_device(l)) != PV_OK) return st;
    const std::vector<double> coef = tp_step_coefficients(a, b, dt, M);
    const TpVjpLayout T{static_cast<char*>(work), vec_bytes(l, dtype, nb), nsteps, M,
                        pv_cheb_propagate_vjp_workspace_size(l, dtype, nb, M, nsteps)};
    return tp_forward_keep(l, dtype, nb, a, b, M, nsteps, coef.data(), psi0, psiT, T, keep_series != 0,
                           static_cast<hipStream_t>(stream));
}

extern "C" pv_status pv_cheb_propagate_vjp_keep(pv_lattice* l, int dtype, int nb, double a, double b, double dt,
                                                int M, int nsteps, const void* psi0, const void* psibar,
                                                void* psi0bar, double* gradV, int keep_series, void* work,
                                                size_t work_bytes, void* stream) {
    pv_status st;
    if ((st = check_tp_vjp_args(l, dtype, nb, a, b, dt, M, nsteps, psi0, psibar, psi0bar, gradV, work, work_bytes,
                                keep_series)) != PV_OK)
        return st;
    return tp_vjp_impl(l, dtype, nb, a, b, dt, M, nsteps, psi0, psibar, psi0bar, gradV, work,
                       static_cast<hipStream_t>(stream), true, keep_series != 0);
}

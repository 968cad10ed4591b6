// Stencil kernels generated at run time from a stencil's own block structure
// (Sec. 3.2: the DSL front end generates the stencil code of a model).
//
// The built-in families (TI, graphene, Weyl) fix their offsets and the zero /
// real / imaginary / complex structure of every block at compile time, so a
// lane's row of every block sits in registers as "slots".  A stencil that
// none of them matches (any DSL program) is described the same way by the
// host -- a pattern struct pv::PatCG with its offsets and entry codes -- and
// the very sweep templates of the built-in families (staged and direct) are
// instantiated for it with hipRTC the first time a launch needs them.  The
// code objects stay loaded for the life of the process, one per device,
// pattern and kernel instance; PV_CODEGEN_CACHE names a directory that keeps
// them across processes.
#include "pv_sweep.hpp"

#include <hip/hiprtc.h>

#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include <unistd.h>

namespace pv {

// Text of pv_kernels.hpp and pv_sweep.hpp, embedded by the build.
extern const char* const kRtcKernelsHpp;
extern const char* const kRtcSweepHpp;

namespace {

thread_local std::string g_err;

// Host stand-in of a generated pattern: the launch set-up (kernel arguments,
// walk and strip layout, LDS size) depends only on the orbitals, the lattice
// dimension and the side rows (x halo, rows at w -+ 1).
template <int NO_, int DIM_, bool SH, bool SW>
struct PatShape {
    static constexpr int FAMILY = FAM_CODEGEN, NO = NO_, NT = 0, DIM = DIM_;
    static constexpr bool SIDE_HALO = SH, SIDE_W = SW;
    static constexpr int off[1][3] = {{0, 0, 0}};
    static constexpr unsigned char code[1][NO_][NO_] = {};
};

struct Compiled {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    int occ = 1;   // workgroups resident per CU at the instance's LDS size
};

std::mutex g_mu;
std::map<std::tuple<int, std::string, std::string>, Compiled> g_fns;   // (device, pattern, instance)

const char* const kOpts[] = {"-O3", "-std=c++17", "-DPV_RTC=1",
                             // keep the compiler from forming packed FP32 instructions
                             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};

uint64_t fnv1a(uint64_t h, const char* s, size_t n) {
    for (size_t i = 0; i < n; ++i) {
        h ^= static_cast<unsigned char>(s[i]);
        h *= 1099511628211ull;
    }
    return h;
}
uint64_t fnv1a(uint64_t h, const std::string& s) { return fnv1a(h, s.data(), s.size() + 1); }

std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "gfx950";
    const std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// Cache file: the kernel's symbol name on the first line, then the code object
// (an ELF file; anything else is a miss).
bool read_cached(const std::string& path, std::string& lowered, std::vector<char>& code) {
    std::ifstream f(path, std::ios::binary);
    if (!f || !std::getline(f, lowered) || lowered.empty()) return false;
    code.assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
    return code.size() > 64 && std::memcmp(code.data(), "\x7f" "ELF", 4) == 0;
}

void write_cached(const std::string& path, const std::string& lowered, const std::vector<char>& code) {
    // a name of this process and call: processes sharing the directory never
    // write one temporary file, and the rename publishes whole files only
    const std::string tmp = path + ".tmp" + std::to_string(static_cast<long>(getpid())) + "_" +
                            std::to_string(reinterpret_cast<uintptr_t>(&code));
    {
        std::ofstream f(tmp, std::ios::binary);
        if (!f) return;
        f << lowered << '\n';
        f.write(code.data(), std::streamsize(code.size()));
        if (!f) return;
    }
    std::rename(tmp.c_str(), path.c_str());
}

// Code object and symbol of the instance `expr` for the pattern; *cached
// says whether they came from the on-disk cache (use_cache: look there).
bool build(const std::string& pat, const std::string& expr, const std::string& arch, bool use_cache,
           std::string& lowered, std::vector<char>& code, bool* cached) {
    const std::string src = "#include \"pv_sweep.hpp\"\n\nnamespace pv {\n\n" + pat + "\n}  // namespace pv\n";
    std::string path;
    *cached = false;
    if (const char* dir = std::getenv("PV_CODEGEN_CACHE"); dir && *dir) {
        uint64_t h = 14695981039346656037ull;
        h = fnv1a(h, arch);
        h = fnv1a(h, src);
        h = fnv1a(h, expr);
        h = fnv1a(h, std::string(kRtcKernelsHpp));
        h = fnv1a(h, std::string(kRtcSweepHpp));
        for (const char* o : kOpts) h = fnv1a(h, std::string(o));
        char name[64];
        std::snprintf(name, sizeof name, "/pvcg_%016llx.co", static_cast<unsigned long long>(h));
        path = std::string(dir) + name;
        if (use_cache && read_cached(path, lowered, code)) {
            *cached = true;
            return true;
        }
    }
    // test hook: PV_TEST_FAIL_CODEGEN=1 makes every compilation fail
    if (const char* f = std::getenv("PV_TEST_FAIL_CODEGEN"); f && std::strcmp(f, "1") == 0) {
        g_err = "hipRTC compile of " + expr + ": failed on request (PV_TEST_FAIL_CODEGEN)";
        return false;
    }
    hiprtcProgram prog;
    const char* hdrs[2] = {kRtcKernelsHpp, kRtcSweepHpp};
    const char* names[2] = {"pv_kernels.hpp", "pv_sweep.hpp"};
    hiprtcResult r = hiprtcCreateProgram(&prog, src.c_str(), "pv_codegen.hip", 2, hdrs, names);
    if (r != HIPRTC_SUCCESS) {
        g_err = std::string("hiprtcCreateProgram: ") + hiprtcGetErrorString(r);
        return false;
    }
    std::vector<const char*> opts;
    const std::string archopt = "--offload-arch=" + arch;
    opts.push_back(archopt.c_str());
    for (const char* o : kOpts) opts.push_back(o);
    if ((r = hiprtcAddNameExpression(prog, expr.c_str())) == HIPRTC_SUCCESS)
        r = hiprtcCompileProgram(prog, int(opts.size()), opts.data());
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        std::string log;
        if (hiprtcGetProgramLogSize(prog, &n) == HIPRTC_SUCCESS && n > 1) {
            log.resize(n);
            if (hiprtcGetProgramLog(prog, &log[0]) != HIPRTC_SUCCESS) log.clear();
        }
        g_err = std::string("hipRTC compile of ") + expr + ": " + hiprtcGetErrorString(r) + "\n" + log.substr(0, 4000);
        (void)hiprtcDestroyProgram(&prog);
        return false;
    }
    const char* lo = nullptr;
    size_t n = 0;
    if (hiprtcGetLoweredName(prog, expr.c_str(), &lo) != HIPRTC_SUCCESS || !lo ||
        hiprtcGetCodeSize(prog, &n) != HIPRTC_SUCCESS || n == 0) {
        g_err = "hipRTC: no code object for " + expr;
        (void)hiprtcDestroyProgram(&prog);
        return false;
    }
    lowered = lo;
    code.resize(n);
    r = hiprtcGetCode(prog, code.data());
    (void)hiprtcDestroyProgram(&prog);
    if (r != HIPRTC_SUCCESS) {
        g_err = std::string("hiprtcGetCode: ") + hiprtcGetErrorString(r);
        return false;
    }
    if (!path.empty()) write_cached(path, lowered, code);
    return true;
}

// The loaded kernel for (current device, pattern, instance), compiled on
// first use (nocompile: hipErrorNotReady instead).  nt and lds: the launch's
// workgroup and LDS size (for the occupancy that sizes staged grids).
hipError_t function_for(const char* pat, const std::string& expr, int nt, size_t lds, bool nocompile,
                        Compiled& out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_mu);
    const auto key = std::make_tuple(dev, std::string(pat), expr);
    const auto it = g_fns.find(key);
    if (it != g_fns.end()) {
        out = it->second;
        return hipSuccess;
    }
    if (nocompile) return hipErrorNotReady;
    g_err.clear();
    const std::string arch = device_arch();
    Compiled c;
    // a cached code object that does not load (a damaged file) is compiled again
    for (int attempt = 0; attempt < 2; ++attempt) {
        std::string lowered;
        std::vector<char> code;
        bool cached = false;
        if (!build(pat, expr, arch, attempt == 0, lowered, code, &cached)) return hipErrorInvalidImage;
        e = hipModuleLoadData(&c.mod, code.data());
        if (e == hipSuccess) {
            e = hipModuleGetFunction(&c.fn, c.mod, lowered.c_str());
            if (e == hipSuccess) break;
            (void)hipModuleUnload(c.mod);
            c.mod = nullptr;
            g_err = "hipModuleGetFunction " + lowered + ": " + hipGetErrorString(e);
        } else {
            g_err = "hipModuleLoadData of " + expr + ": " + hipGetErrorString(e);
        }
        if (!cached) return e;
        (void)hipGetLastError();
    }
    if (e != hipSuccess) return e;
    g_err.clear();
    int n = 0;
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&n, c.fn, nt, lds) != hipSuccess || n < 1) n = 1;
    c.occ = n;
    g_fns.emplace(key, c);
    out = c;
    return hipSuccess;
}

// LDS bytes a workgroup may use on the current device (asked once per device).
size_t max_lds() {
    static std::mutex mu;
    static std::map<int, size_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    std::lock_guard<std::mutex> lk(mu);
    const auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) v = 65536;
    cache[dev] = size_t(v);
    return size_t(v);
}

template <typename T>
const char* tname() {
    return sizeof(T) == 8 ? "double" : "float";
}

// Staged sweep of E elements per lane, NT lanes, epilogue flags epm (0: read
// at run time): the set-up of launch_staged with the generated kernel.
template <class P, typename T, typename VT, int E, int NT>
hipError_t staged_go(SweepParams& p, int num_cus, hipStream_t s, unsigned epm) {
    KArgs<T, VT> a;
    make_kargs<P, T, VT>(p, false, a);
    const size_t lds = staged_lds_bytes_for<P, T, E, NT>(epm == 0u || (epm & EP_ACC_ADD) != 0u);
    char expr[160];
    std::snprintf(expr, sizeof expr, "&pv::staged_kernel<pv::PatCG, %s, %s, %d, %uu, %d>", tname<T>(), tname<VT>(),
                  E, epm, NT);
    Compiled c;
    if (const hipError_t e = function_for(p.cg_src, expr, NT, lds, p.cg_nocompile != 0, c); e != hipSuccess) return e;
    int G8 = p.st_G8 > 0 ? p.st_G8 : (num_cus >= 8 ? num_cus / 8 : 1) * c.occ;
    if (G8 > 256) G8 = 256;
    G8 = staged_setup<P, T, VT, E, NT>(p, G8, false, a);
    p.grid = 8 * G8;
    void* args[] = {&a};
    return hipModuleLaunchKernel(c.fn, unsigned(p.grid), 1, 1, NT, 1, 1, unsigned(lds), s, args, nullptr);
}

// Epilogue specialisations as for the built-in families: the Chebyshev step
// with dots, the series step and the plain sweep (without z when gamma = 0)
// with uniform alpha, beta, gamma; everything else reads its flags at run
// time (complex128: one element per lane).
template <class P, typename T, typename VT, int E>
hipError_t staged_ep(SweepParams& p, int num_cus, hipStream_t s) {
    constexpr unsigned KPM = EP_STORE_Y | EP_DOTS, SERIES = EP_STORE_Y | EP_ACC_ADD, PLAIN = EP_STORE_Y;
    constexpr int E0 = sizeof(T) == 8 ? 1 : 2;
    if constexpr (E != E0) {
        // a tile whose rows (six side rows with SIDE_W) overflow the CU's LDS
        // takes the shortest tile instead
        if (staged_lds_bytes_for<P, T, E, kBlock>(true) > max_lds() ||
            (p.st_nt == 512 && staged_lds_bytes_for<P, T, E, 512>(true) > max_lds()))
            return staged_ep<P, T, VT, E0>(p, num_cus, s);
    }
    if (p.colp == nullptr) {
        unsigned epm = 0u;
        if (p.ep == KPM) epm = KPM;
        else if (p.ep == SERIES) epm = SERIES;
        else if (p.ep == PLAIN) epm = p.gamma == 0.0 ? (PLAIN | EP_NO_Z) : PLAIN;
        if (epm != 0u) {
            if (p.st_nt == 512 && staged_lds_bytes_for<P, T, E, 512>(true) <= max_lds())
                return staged_go<P, T, VT, E, 512>(p, num_cus, s, epm);
            return staged_go<P, T, VT, E, kBlock>(p, num_cus, s, epm);
        }
    }
    if constexpr (sizeof(T) == 8 && E == 2) {
        SweepParams q = p;
        q.st_C = q.st_Bm = q.st_G8 = 0;
        const hipError_t e = staged_go<P, T, VT, 1, kBlock>(q, num_cus, s, 0u);
        p.grid = q.grid;
        return e;
    } else {
        return staged_go<P, T, VT, E, kBlock>(p, num_cus, s, 0u);
    }
}

// Kernel choice of a built-in family: staged when the block is 16-byte
// aligned in whole chunks per site and the launch asks for it or is large
// (every generated pattern stages: 3D stencils with hops that have a y and a
// z step take six side rows, (m -+ 1, w) and (m -+ 1, w -+ 1)); else the
// direct kernel.
template <class P, typename T, typename VT>
hipError_t typed(SweepParams& p, int num_cus, hipStream_t s) {
    static const int env_kernel = env_int("PV_SWEEP", 0);
    const int kind = p.kernel > 0 ? p.kernel : env_kernel;
    const bool aligned = ((reinterpret_cast<uintptr_t>(p.x) | reinterpret_cast<uintptr_t>(p.zero_row)) & 15) == 0;
    const bool whole = (P::NO * p.nb * int(sizeof(cplx<T>))) % 16 == 0;
    if (aligned && whole && P::NO * p.nb <= STAGED_MAX_SITE && (kind == 2 || (kind == 0 && staged_default(p)))) {
        const int e = staged_elems(p);
        if constexpr (sizeof(T) == 8)
            return e == 2 ? staged_ep<P, T, VT, 2>(p, num_cus, s) : staged_ep<P, T, VT, 1>(p, num_cus, s);
        else
            return e == 4 ? staged_ep<P, T, VT, 4>(p, num_cus, s) : staged_ep<P, T, VT, 2>(p, num_cus, s);
    }
    KArgs<T, VT> a;
    make_kargs<P, T, VT>(p, false, a);
    p.grid = int(8 * ((a.ntiles + a.tpb - 1) / a.tpb));
    char expr[128];
    std::snprintf(expr, sizeof expr, "&pv::sweep_kernel<pv::PatCG, %s, %s>", tname<T>(), tname<VT>());
    Compiled c;
    if (const hipError_t e = function_for(p.cg_src, expr, kBlock, 0, p.cg_nocompile != 0, c); e != hipSuccess) return e;
    void* args[] = {&a};
    return hipModuleLaunchKernel(c.fn, unsigned(p.grid), 1, 1, kBlock, 1, 1, 0, s, args, nullptr);
}

// Calls f(Tag<P>, Tag<T>, Tag<VT>) with the host stand-in of the launch's
// pattern and its vector and field types.
template <class F>
hipError_t with_pattern(const SweepParams& p, F&& f) {
    auto types = [&](auto pt) -> hipError_t {
        using P = typename decltype(pt)::type;
        if (p.dtype == 0) {
            if (p.vtype != 0) return hipErrorInvalidValue;
            return f(Tag<P>{}, Tag<double>{}, Tag<double>{});
        }
        if (p.vtype == 0) return f(Tag<P>{}, Tag<float>{}, Tag<double>{});
        return f(Tag<P>{}, Tag<float>{}, Tag<float>{});
    };
    auto shape = [&](auto no) -> hipError_t {
        constexpr int NO = decltype(no)::value;
        if (p.cg_dim == 2) return types(Tag<PatShape<NO, 2, false, false>>{});
        if (p.cg_sidew)
            return p.cg_halo ? types(Tag<PatShape<NO, 3, true, true>>{}) : types(Tag<PatShape<NO, 3, false, true>>{});
        return p.cg_halo ? types(Tag<PatShape<NO, 3, true, false>>{}) : types(Tag<PatShape<NO, 3, false, false>>{});
    };
    switch (p.n_orb) {
        case 1: return shape(IntC<1>{});
        case 2: return shape(IntC<2>{});
        case 4: return shape(IntC<4>{});
        default: return hipErrorInvalidValue;
    }
}

// Elements per lane and lanes of a batched staged launch (the Chebyshev step
// with dots): the batch's shape, or the shortest tile where the LDS would
// overflow; calls g(IntC<E>, IntC<NT>).
template <class P, typename T, class G>
hipError_t batch_tile(const SweepParams& p, G&& g) {
    constexpr int E0 = sizeof(T) == 8 ? 1 : 2, E1 = 2 * E0;
    const int e = staged_elems(p);
    const bool w512 = p.st_nt == 512;
    auto fits = [](size_t lds) { return lds <= max_lds(); };
    if (e == E1) {
        if (w512 && fits(staged_lds_bytes_for<P, T, E1, 512>(false))) return g(IntC<E1>{}, IntC<512>{});
        if (!w512 && fits(staged_lds_bytes_for<P, T, E1, kBlock>(false))) return g(IntC<E1>{}, IntC<kBlock>{});
    }
    if (w512 && fits(staged_lds_bytes_for<P, T, E0, 512>(false))) return g(IntC<E0>{}, IntC<512>{});
    return g(IntC<E0>{}, IntC<kBlock>{});
}

}  // namespace

hipError_t launch_codegen(SweepParams& p, int num_cus, hipStream_t s) {
    g_err.clear();
    if (!p.cg_src) return hipErrorInvalidValue;
    return with_pattern(p, [&](auto pt, auto tt, auto vt) -> hipError_t {
        return typed<typename decltype(pt)::type, typename decltype(tt)::type, typename decltype(vt)::type>(
            p, num_cus, s);
    });
}

// Batched sweeps (one launch per step over every instance of a batch whose
// lattices share one generated pattern): argument records and launches as
// for the built-in families.
hipError_t codegen_batch_fill_record(const SweepParams& p, int staged, void* dst, int* nblocks) {
    return with_pattern(p, [&](auto pt, auto tt, auto vt) -> hipError_t {
        using P = typename decltype(pt)::type;
        using T = typename decltype(tt)::type;
        using VT = typename decltype(vt)::type;
        static_assert(sizeof(KArgs<T, VT>) == sizeof(KArgs<double, double>), "record sizes differ");
        KArgs<T, VT> a;
        if (staged) {
            if (P::NO * p.nb > STAGED_MAX_SITE || (P::NO * p.nb * int(sizeof(cplx<T>))) % 16 != 0)
                return hipErrorInvalidValue;
            make_kargs<P, T, VT>(p, false, a);
            return batch_tile<P, T>(p, [&](auto ke, auto kn) -> hipError_t {
                const int G8 = staged_setup<P, T, VT, decltype(ke)::value, decltype(kn)::value>(p, 1 << 30, true, a);
                std::memcpy(dst, &a, sizeof(a));
                *nblocks = 8 * G8;
                return hipSuccess;
            });
        }
        make_kargs<P, T, VT>(p, true, a);
        std::memcpy(dst, &a, sizeof(a));
        *nblocks = int((a.ntiles + a.tpb - 1) / a.tpb);
        return hipSuccess;
    });
}

namespace {

// The batched kernel instance of a launch and its LDS bytes, loaded (and
// compiled on first use unless nocompile).
hipError_t batch_function(const SweepParams& p, int staged, bool nocompile, Compiled& c, int& nt, size_t& lds) {
    return with_pattern(p, [&](auto pt, auto tt, auto vt) -> hipError_t {
        using P = typename decltype(pt)::type;
        using T = typename decltype(tt)::type;
        using VT = typename decltype(vt)::type;
        char expr[160];
        if (!staged) {
            std::snprintf(expr, sizeof expr, "&pv::batch_sweep_kernel<pv::PatCG, %s, %s>", tname<T>(), tname<VT>());
            nt = kBlock;
            lds = 0;
            return function_for(p.cg_src, expr, kBlock, 0, nocompile, c);
        }
        return batch_tile<P, T>(p, [&](auto ke, auto kn) -> hipError_t {
            constexpr int E = decltype(ke)::value, NT = decltype(kn)::value;
            std::snprintf(expr, sizeof expr, "&pv::batch_staged_kernel<pv::PatCG, %s, %s, %d, %uu, %d>", tname<T>(),
                          tname<VT>(), E, unsigned(EP_STORE_Y | EP_DOTS), NT);
            nt = NT;
            lds = staged_lds_bytes_for<P, T, E, NT>(false);
            return function_for(p.cg_src, expr, NT, lds, nocompile, c);
        });
    });
}

}  // namespace

hipError_t codegen_prepare_batch(const SweepParams& p, int staged) {
    g_err.clear();
    Compiled c;
    int nt = 0;
    size_t lds = 0;
    return batch_function(p, staged, false, c, nt, lds);
}

hipError_t launch_batch_codegen(const SweepParams& p, int staged, const void* table, const int* block_inst,
                                const int* inst_block0, int grid, int red_step, hipStream_t s) {
    g_err.clear();
    if (staged && p.ep != (EP_STORE_Y | EP_DOTS)) return hipErrorInvalidValue;
    Compiled c;
    int nt = 0;
    size_t lds = 0;
    if (const hipError_t e = batch_function(p, staged, false, c, nt, lds); e != hipSuccess) return e;
    void* args[] = {&table, &block_inst, &inst_block0, &red_step};
    return hipModuleLaunchKernel(c.fn, unsigned(grid), 1, 1, unsigned(nt), 1, 1, unsigned(lds), s, args, nullptr);
}

const char* codegen_error() { return g_err.c_str(); }

int codegen_instances() {
    std::lock_guard<std::mutex> lk(g_mu);
    return int(g_fns.size());
}
void codegen_clear_error() { g_err.clear(); }

}  // namespace pv

// Front end for the stencil description language of Sec. 3.2: the text of a
// DSL program becomes the lattice descriptor arrays of pv_lattice_create.
//
// Accepted text (one statement per line; blank lines and lines starting with
// '#' are skipped):
//   dim D                       2 or 3
//   size S                      orbitals per site, 1..PV_MAX_ORB
//   n_coeff_const N             number of constant coefficients (type c)
//   n_coeff_variable N          number of per-site variable coefficients (v)
//   n_coeff_rand N              number of per-site random coefficients (r)
//   coeff_const_default v...    default values of the constant coefficients
//   nn d0 d1 [d2]               a block at offset d = (d0, d1, d2) along
//                               (x, y, z), followed by exactly S row lines
// Row line k:  [l<k>;] entry; entry; ...   (empty entries allowed; a row
//              without entries is written as its label, e.g. "l2;"; blank
//              and comment lines inside a block are skipped)
// Entry:       col|value  or  col|type|arg, type f (fixed, arg = value),
//              c (arg = index into the constant coefficients), v or r
//              (arg = index of the per-site coefficient).
// Values are reals, or complex as <re>i, <re>+<im>i, <re>-<im>i (an
// extension: the tight-binding blocks of Sec. 2.2 are complex).
//
// Meaning: entry (row k, column q) of the block at offset d adds
// value * x[s + d][q] to y[s][k] -- the descriptor convention of the library.
// Per-site coefficients (v, r) may only sit on the diagonal of the on-site
// block (nn 0 0 ...), where they add to a fixed or constant entry of the same
// position if there is one: one index for every orbital gives a per-site field
// (PV_POT_SITE), index k on row k a per-orbital field (PV_POT_ORBITAL); v
// fields are attached with pv_lattice_set_potential, r fields are generated
// on the fly (pv_lattice_set_random_potential).
#include <cctype>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <sstream>
#include <string>
#include <vector>

#include "pvdtm.h"

// error reporting of the C ABI (pv_api.cpp)
pv_status pv_fail_status(pv_status st, const char* msg);

namespace {

using cd = std::complex<double>;

pv_status dsl_fail(int line, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    char msg[600];
    std::snprintf(msg, sizeof msg, "DSL line %d: %s", line, buf);
    return pv_fail_status(PV_ERR_INVALID_ARG, msg);
}

std::string trim(const std::string& s) {
    size_t a = 0, b = s.size();
    while (a < b && std::isspace((unsigned char)s[a])) ++a;
    while (b > a && std::isspace((unsigned char)s[b - 1])) --b;
    return s.substr(a, b - a);
}

std::vector<std::string> split(const std::string& s, char sep) {
    std::vector<std::string> out;
    std::string cur;
    for (char ch : s) {
        if (ch == sep) {
            out.push_back(cur);
            cur.clear();
        } else {
            cur += ch;
        }
    }
    out.push_back(cur);
    return out;
}

bool parse_int(const std::string& t, long long& v) {
    const std::string s = trim(t);
    if (s.empty()) return false;
    char* end = nullptr;
    v = std::strtoll(s.c_str(), &end, 10);
    return end && *end == '\0';
}

bool parse_real(const std::string& s, double& v) {
    if (s.empty()) return false;
    char* end = nullptr;
    v = std::strtod(s.c_str(), &end);
    return end && *end == '\0' && std::isfinite(v);
}

// real, <im>i, <re>+<im>i, <re>-<im>i
bool parse_value(const std::string& t, cd& v) {
    const std::string s = trim(t);
    if (s.empty()) return false;
    if (s.back() != 'i') {
        double r;
        if (!parse_real(s, r)) return false;
        v = cd(r, 0.0);
        return true;
    }
    const std::string body = s.substr(0, s.size() - 1);
    // split at the last sign that is not the first character and not part of an exponent
    size_t cut = std::string::npos;
    for (size_t k = body.size(); k-- > 1;)
        if ((body[k] == '+' || body[k] == '-') && body[k - 1] != 'e' && body[k - 1] != 'E') {
            cut = k;
            break;
        }
    double re = 0.0, im = 0.0;
    if (cut == std::string::npos) {
        if (body.empty() || body == "+") im = 1.0;
        else if (body == "-") im = -1.0;
        else if (!parse_real(body, im)) return false;
    } else {
        if (!parse_real(body.substr(0, cut), re)) return false;
        const std::string ip = body.substr(cut);
        if (ip == "+") im = 1.0;
        else if (ip == "-") im = -1.0;
        else if (!parse_real(ip, im)) return false;
    }
    v = cd(re, im);
    return true;
}

struct Block {
    int off[3] = {0, 0, 0};
    std::vector<cd> m;              // [S][S] fixed and constant entries
    std::vector<int> set;           // entry present
    std::vector<int> site_kind;     // diagonal only: 0 none, 'v' or 'r'
    std::vector<int> site_index;
};

}  // namespace

extern "C" pv_status pv_dsl_stencil(const char* text, const double* coeff_const, int n_const, int* dim,
                                    int* n_orb, int* n_terms, int* offsets, double* blocks, double* onsite,
                                    int* pot_mode, int* field_kind) {
    if (!text || !dim || !n_orb || !n_terms || !offsets || !blocks || !onsite || !pot_mode)
        return pv_fail_status(PV_ERR_INVALID_ARG, "pv_dsl_stencil: NULL argument");
    if (n_const < 0 || (n_const > 0 && !coeff_const))
        return pv_fail_status(PV_ERR_INVALID_ARG, "pv_dsl_stencil: coeff_const array missing");
    std::vector<std::string> lines;
    {
        std::string all(text), cur;
        for (char ch : all) {
            if (ch == '\n') {
                lines.push_back(cur);
                cur.clear();
            } else if (ch != '\r') {
                cur += ch;
            }
        }
        lines.push_back(cur);
    }
    int D = 0, S = 0;
    long long nc = 0, nv = 0, nr = 0;
    std::vector<cd> cdef;
    std::vector<Block> blks;
    for (size_t li = 0; li < lines.size(); ++li) {
        const int ln = int(li + 1);
        const std::string line = trim(lines[li]);
        if (line.empty() || line[0] == '#') continue;
        std::istringstream is(line);
        std::string kw;
        is >> kw;
        std::vector<std::string> args;
        for (std::string a; is >> a;) args.push_back(a);
        auto one_int = [&](long long& v, long long lo, long long hi) -> pv_status {
            if (args.size() != 1 || !parse_int(args[0], v) || v < lo || v > hi)
                return dsl_fail(ln, "'%s' needs one integer in [%lld, %lld]", kw.c_str(), lo, hi);
            return PV_OK;
        };
        pv_status st = PV_OK;
        long long v = 0;
        if (kw == "dim") {
            if ((st = one_int(v, 2, 3)) != PV_OK) return st;
            if (D) return dsl_fail(ln, "'dim' given twice");
            D = int(v);
        } else if (kw == "size") {
            if ((st = one_int(v, 1, PV_MAX_ORB)) != PV_OK) return st;
            if (S) return dsl_fail(ln, "'size' given twice");
            S = int(v);
        } else if (kw == "n_coeff_const") {
            if ((st = one_int(nc, 0, 1 << 20)) != PV_OK) return st;
        } else if (kw == "n_coeff_variable") {
            if ((st = one_int(nv, 0, 1 << 20)) != PV_OK) return st;
        } else if (kw == "n_coeff_rand") {
            if ((st = one_int(nr, 0, 1 << 20)) != PV_OK) return st;
        } else if (kw == "coeff_const_default") {
            cdef.clear();
            for (const auto& a : args) {
                cd c;
                if (!parse_value(a, c)) return dsl_fail(ln, "bad value '%s'", a.c_str());
                cdef.push_back(c);
            }
        } else if (kw == "nn") {
            if (!D || !S) return dsl_fail(ln, "'dim' and 'size' must precede the first 'nn'");
            if ((int)args.size() != D) return dsl_fail(ln, "'nn' needs %d offsets for dim %d", D, D);
            Block b;
            for (int d = 0; d < D; ++d) {
                long long o;
                if (!parse_int(args[d], o) || o < -1 || o > 1) return dsl_fail(ln, "offsets must be -1, 0 or 1");
                b.off[d] = int(o);
            }
            for (const Block& q : blks)
                if (q.off[0] == b.off[0] && q.off[1] == b.off[1] && q.off[2] == b.off[2])
                    return dsl_fail(ln, "offset (%d, %d, %d) defined twice", b.off[0], b.off[1], b.off[2]);
            const bool onsite_blk = !b.off[0] && !b.off[1] && !b.off[2];
            b.m.assign(S * S, cd(0, 0));
            b.set.assign(S * S, 0);
            b.site_kind.assign(S, 0);
            b.site_index.assign(S, -1);
            // the S row lines (skipping blank and comment lines)
            for (int row = 0; row < S; ++row) {
                size_t lj = li + 1;
                while (lj < lines.size() && (trim(lines[lj]).empty() || trim(lines[lj])[0] == '#')) ++lj;
                if (lj >= lines.size()) return dsl_fail(ln, "block ends after %d of %d rows", row, S);
                li = lj;
                const int rln = int(li + 1);
                std::vector<std::string> fields = split(lines[li], ';');
                size_t f0 = 0;
                const std::string first = trim(fields[0]);
                if (!first.empty() && first[0] == 'l') {
                    long long k;
                    if (!parse_int(first.substr(1), k) || k != row)
                        return dsl_fail(rln, "row label '%s' where l%d was expected", first.c_str(), row);
                    f0 = 1;
                } else if (!first.empty() && first.find('|') == std::string::npos) {
                    return dsl_fail(rln, "'%s' is neither a row label nor an entry", first.c_str());
                }
                for (size_t f = f0; f < fields.size(); ++f) {
                    const std::string e = trim(fields[f]);
                    if (e.empty()) continue;
                    std::vector<std::string> parts = split(e, '|');
                    long long col;
                    if (parts.size() < 2 || parts.size() > 3 || !parse_int(parts[0], col) || col < 0 || col >= S)
                        return dsl_fail(rln, "bad entry '%s' (col|value or col|type|arg, col < %d)", e.c_str(), S);
                    const int idx = row * S + int(col);
                    std::string type = parts.size() == 3 ? trim(parts[1]) : "f";
                    // a diagonal position may hold one fixed / constant entry and
                    // one per-site entry (they add); anything else only once
                    const bool per_site = type == "v" || type == "r";
                    if (per_site ? b.site_kind[row] != 0 : b.set[idx] != 0)
                        return dsl_fail(rln, "entry (%d, %lld) given twice", row, col);
                    if (!per_site) b.set[idx] = 1;
                    const std::string arg = trim(parts.back());
                    if (type == "f") {
                        cd c;
                        if (!parse_value(arg, c)) return dsl_fail(rln, "bad value '%s'", arg.c_str());
                        b.m[idx] = c;
                    } else if (type == "c") {
                        long long k;
                        if (!parse_int(arg, k) || k < 0 || k >= nc)
                            return dsl_fail(rln, "constant index '%s' outside n_coeff_const = %lld", arg.c_str(), nc);
                        cd c;
                        if (k < n_const) c = cd(coeff_const[k], 0.0);
                        else if (k < (long long)cdef.size()) c = cdef[k];
                        else return dsl_fail(rln, "constant %lld has no value (coeff_const_default)", k);
                        b.m[idx] = c;
                    } else if (type == "v" || type == "r") {
                        long long k;
                        const long long n = type == "v" ? nv : nr;
                        if (!parse_int(arg, k) || k < 0 || k >= n)
                            return dsl_fail(rln, "%s index '%s' outside n_coeff_%s = %lld", type.c_str(), arg.c_str(),
                                            type == "v" ? "variable" : "rand", n);
                        if (!onsite_blk || col != row)
                            return dsl_fail(rln, "per-site coefficients are supported on the on-site diagonal only");
                        b.site_kind[row] = type[0];
                        b.site_index[row] = int(k);
                    } else {
                        return dsl_fail(rln, "unknown coefficient type '%s' (f, c, v, r)", type.c_str());
                    }
                }
            }
            blks.push_back(b);
        } else {
            return dsl_fail(ln, "unknown statement '%s'", kw.c_str());
        }
    }
    if (!D || !S) return pv_fail_status(PV_ERR_INVALID_ARG, "DSL: 'dim' and 'size' are required");

    // assemble the descriptor
    int nt = 0, pm = PV_POT_NONE, fk = 0;
    for (int k = 0; k < S * S * 2; ++k) onsite[k] = 0.0;
    for (const Block& b : blks) {
        const bool onsite_blk = !b.off[0] && !b.off[1] && !b.off[2];
        if (onsite_blk) {
            for (int k = 0; k < S * S; ++k) {
                onsite[2 * k] = b.m[k].real();
                onsite[2 * k + 1] = b.m[k].imag();
            }
            int kinds = 0, same = 1, diag = 1, any = 0;
            for (int r = 0; r < S; ++r) {
                if (b.site_kind[r]) {
                    any = 1;
                    kinds |= (b.site_kind[r] == 'v') ? 1 : 2;
                    if (b.site_index[r] != b.site_index[0]) same = 0;
                    if (b.site_index[r] != r) diag = 0;
                }
            }
            if (any) {
                for (int r = 0; r < S; ++r)
                    if (!b.site_kind[r])
                        return pv_fail_status(PV_ERR_UNSUPPORTED,
                                              "DSL: per-site coefficients must cover every orbital of the diagonal");
                if (kinds == 3)
                    return pv_fail_status(PV_ERR_UNSUPPORTED, "DSL: v and r coefficients on one diagonal");
                if (same) pm = PV_POT_SITE;
                else if (diag) pm = PV_POT_ORBITAL;
                else
                    return pv_fail_status(PV_ERR_UNSUPPORTED,
                                          "DSL: per-site diagonal indices must be all equal or equal to the row");
                fk = (kinds == 1) ? 1 : 2;
            }
            continue;
        }
        if (nt >= PV_MAX_TERMS) return pv_fail_status(PV_ERR_UNSUPPORTED, "DSL: too many neighbour blocks");
        for (int d = 0; d < 3; ++d) offsets[3 * nt + d] = b.off[d];
        for (int k = 0; k < S * S; ++k) {
            blocks[(size_t)(nt * S * S + k) * 2] = b.m[k].real();
            blocks[(size_t)(nt * S * S + k) * 2 + 1] = b.m[k].imag();
        }
        ++nt;
    }
    *dim = D;
    *n_orb = S;
    *n_terms = nt;
    *pot_mode = pm;
    if (field_kind) *field_kind = fk;
    return PV_OK;
}

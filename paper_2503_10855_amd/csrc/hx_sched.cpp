// hx_sched.cpp -- a small scheduling language for the EDGE fork-joins.
//
// The algorithm is fixed: six fork-joins over [H, W] (blur, laplacian,
// zero_cross, sobel, the max reduction max_gradient, threshold), each
// initially its own kernel, with max_gradient a sequential reduction.  A
// schedule is a list of statements applying transformations to labels,
// in the manner of the Juno scheduling language (The Juno Scheduling
// Language; the reduction_tree macro of Use and Impact of Schedules):
//
//   fork-tile[rows, cols](labels)   tile the kernel holding the labels
//   fork-fuse(labels)               fuse the kernels holding the labels
//   fork-chunk[N](max_gradient)     chunk the reduction into N parts
//   fork-reshape[...](max_gradient) accepted (chunking already puts the
//                                   chunk loop outside)
//   monoid-reassociate(max_gradient)  start every chunk at the identity
//   fork-fission(max_gradient)      split the chunked loop into a parallel
//                                   fork of partials and a serial combine
//   reduction_tree![N](max_gradient)  the four steps above
//   warp-reduce(max_gradient)       reduce with wave64 primitives and one
//                                   atomic per wave (implies the tree)
//   pass[store|recompute|speculate](threshold)  how a fully fused sweep
//                                   is split around the max it waits for
//
// The transformed program is then lowered onto the kernels that exist
// (hx_schedule); a program with no matching kernel is rejected with the
// reason.  Statements end with ';'; '#' starts a comment; a leading
// "let (names) =" is accepted and ignored.
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hx.h"
#include "hx_kernels.h"
#include "hx_pipeline.h"

namespace hx {
namespace {

enum Stage { BLUR, LAPLACIAN, ZERO_CROSS, SOBEL, MAX_GRADIENT, THRESHOLD, NSTAGES };
const char* const kStageNames[NSTAGES] = {"blur",  "laplacian",    "zero_cross",
                                          "sobel", "max_gradient", "threshold"};

struct Program {
    int group[NSTAGES];     // kernel group of each stage (initially its own)
    int rows[NSTAGES] = {}, cols[NSTAGES] = {};  // tile per group id (0 = unset)
    int chunks = 0;         // fork-chunk factor of max_gradient (0 = none)
    bool reassociated = false, fissioned = false, warp = false;
    int pass = HX_PASS_STORE;
    bool pass_set = false;
};

struct Stmt {
    std::string op;
    bool bang = false;  // macro form (name!), same meaning here
    std::vector<std::string> args;
    std::vector<int> labels;
};

struct Lexer {
    const char* p;
    int stmt_no = 0;
    void skip() {
        for (;;) {
            while (*p && std::isspace((unsigned char)*p)) ++p;
            if (*p == '#') {
                while (*p && *p != '\n') ++p;
                continue;
            }
            return;
        }
    }
    bool word(std::string& out) {
        skip();
        const char* s = p;
        while (*p && (std::isalnum((unsigned char)*p) || *p == '_' || *p == '-')) ++p;
        out.assign(s, p - s);
        return !out.empty();
    }
    bool take(char c) {
        skip();
        if (*p != c) return false;
        ++p;
        return true;
    }
    // A bracketed argument such as fork-reshape's [[0], [1]]: kept as text.
    bool group(std::string& out) {
        skip();
        if (*p != '[') return false;
        const char* s = p;
        int depth = 0;
        do {
            if (*p == '[') ++depth;
            if (*p == ']') --depth;
            ++p;
        } while (*p && depth > 0);
        if (depth) return false;
        out.assign(s, p - s);
        return true;
    }
};

hx_status parse(const char* text, std::vector<Stmt>& out) {
    Lexer lx{text};
    for (;;) {
        lx.skip();
        if (!*lx.p) return HX_OK;
        ++lx.stmt_no;
        Stmt st;
        if (!lx.word(st.op)) return fail(HX_E_INVALID, "statement %d: expected a name", lx.stmt_no);
        if (st.op == "let") {
            // let (a, b) = transformation(...): the names bind the pieces a
            // transformation returns; the labels here are fixed, so they are
            // read and dropped.
            while (*lx.p && *lx.p != '=' && *lx.p != ';') ++lx.p;
            if (!lx.take('=') || !lx.word(st.op))
                return fail(HX_E_INVALID, "statement %d: expected 'let (...) = name(...)'",
                            lx.stmt_no);
        }
        st.bang = lx.take('!');
        if (lx.take('[')) {
            std::string a;
            do {
                if (!lx.word(a) && !lx.group(a))
                    return fail(HX_E_INVALID, "statement %d (%s): bad argument", lx.stmt_no,
                                st.op.c_str());
                st.args.push_back(a);
            } while (lx.take(','));
            if (!lx.take(']'))
                return fail(HX_E_INVALID, "statement %d (%s): expected ']'", lx.stmt_no,
                            st.op.c_str());
        }
        if (!lx.take('('))
            return fail(HX_E_INVALID, "statement %d (%s): expected '('", lx.stmt_no, st.op.c_str());
        std::string l;
        do {
            if (!lx.word(l))
                return fail(HX_E_INVALID, "statement %d (%s): expected a label", lx.stmt_no,
                            st.op.c_str());
            int id = -1;
            for (int i = 0; i < NSTAGES; ++i)
                if (l == kStageNames[i]) id = i;
            if (id < 0)
                return fail(HX_E_INVALID, "statement %d (%s): unknown label '%s'", lx.stmt_no,
                            st.op.c_str(), l.c_str());
            st.labels.push_back(id);
        } while (lx.take(','));
        if (!lx.take(')') || !lx.take(';'))
            return fail(HX_E_INVALID, "statement %d (%s): expected ');'", lx.stmt_no,
                        st.op.c_str());
        out.push_back(std::move(st));
    }
}

bool to_int(const std::string& s, int* v) {
    char* end = nullptr;
    const long x = std::strtol(s.c_str(), &end, 10);
    if (s.empty() || *end || x <= 0 || x > (1 << 20)) return false;
    *v = (int)x;
    return true;
}

hx_status apply(Program& pr, const Stmt& st, int n) {
    auto only_max = [&]() -> hx_status {
        if (st.labels.size() != 1 || st.labels[0] != MAX_GRADIENT)
            return fail(HX_E_INVALID, "statement %d: %s applies to the reduction max_gradient",
                        n, st.op.c_str());
        return HX_OK;
    };
    hx_status s = HX_OK;
    if (st.op == "fork-tile") {
        int r = 0, c = 0;
        if (st.args.size() != 2 || !to_int(st.args[0], &r) || !to_int(st.args[1], &c))
            return fail(HX_E_INVALID, "statement %d: fork-tile takes [rows, cols]", n);
        for (int l : st.labels) {
            if (l == MAX_GRADIENT || l == THRESHOLD)
                return fail(HX_E_INVALID, "statement %d: %s keeps its own launch shape", n,
                            kStageNames[l]);
            pr.rows[pr.group[l]] = r;
            pr.cols[pr.group[l]] = c;
        }
    } else if (st.op == "fork-fuse") {
        if (st.labels.size() < 2)
            return fail(HX_E_INVALID, "statement %d: fork-fuse needs two labels", n);
        const int g = pr.group[st.labels[0]];
        for (int l : st.labels) {
            if (l == MAX_GRADIENT || l == THRESHOLD)
                return fail(HX_E_INVALID,
                            "statement %d: %s depends on the whole image and cannot be fused "
                            "into a stencil kernel",
                            n, kStageNames[l]);
            const int h = pr.group[l];
            if (h == g) continue;
            for (int i = 0; i < NSTAGES; ++i)
                if (pr.group[i] == h) pr.group[i] = g;
            if (!pr.rows[g]) {
                pr.rows[g] = pr.rows[h];
                pr.cols[g] = pr.cols[h];
            }
        }
    } else if (st.op == "fork-chunk") {
        if ((s = only_max()) != HX_OK) return s;
        int c = 0;
        if (st.args.size() != 1 || !to_int(st.args[0], &c))
            return fail(HX_E_INVALID, "statement %d: fork-chunk takes [N]", n);
        pr.chunks = c;
    } else if (st.op == "fork-reshape") {
        if ((s = only_max()) != HX_OK) return s;
        if (!pr.chunks)
            return fail(HX_E_INVALID, "statement %d: fork-reshape needs a chunked loop", n);
    } else if (st.op == "monoid-reassociate") {
        if ((s = only_max()) != HX_OK) return s;
        if (!pr.chunks)
            return fail(HX_E_INVALID, "statement %d: monoid-reassociate needs a chunked loop", n);
        pr.reassociated = true;  // max is a monoid (MonoidReduce)
    } else if (st.op == "fork-fission") {
        if ((s = only_max()) != HX_OK) return s;
        if (!pr.reassociated)
            return fail(HX_E_INVALID,
                        "statement %d: fork-fission of the reduction needs partials that "
                        "start at the identity (monoid-reassociate)",
                        n);
        pr.fissioned = true;
    } else if (st.op == "reduction_tree") {
        if ((s = only_max()) != HX_OK) return s;
        int c = 0;
        if (st.args.size() != 1 || !to_int(st.args[0], &c))
            return fail(HX_E_INVALID, "statement %d: reduction_tree! takes [N]", n);
        pr.chunks = c;
        pr.reassociated = pr.fissioned = true;
    } else if (st.op == "warp-reduce") {
        if ((s = only_max()) != HX_OK) return s;
        pr.warp = true;
    } else if (st.op == "pass") {
        if (st.labels.size() != 1 || st.labels[0] != THRESHOLD || st.args.size() != 1)
            return fail(HX_E_INVALID, "statement %d: pass[store|recompute|speculate](threshold)",
                        n);
        const std::string& a = st.args[0];
        if (a == "store") pr.pass = HX_PASS_STORE;
        else if (a == "recompute") pr.pass = HX_PASS_RECOMPUTE;
        else if (a == "speculate") pr.pass = HX_PASS_SPECULATE;
        else return fail(HX_E_INVALID, "statement %d: unknown pass structure '%s'", n, a.c_str());
        pr.pass_set = true;
    } else {
        return fail(HX_E_INVALID, "statement %d: unknown transformation '%s'", n, st.op.c_str());
    }
    return HX_OK;
}

bool same_group(const Program& pr, std::initializer_list<int> a) {
    const int g = pr.group[*a.begin()];
    for (int x : a)
        if (pr.group[x] != g) return false;
    return true;
}

hx_status lower(const Program& pr, hx_schedule* out) {
    const bool bs = same_group(pr, {BLUR, SOBEL});
    const bool lz = same_group(pr, {LAPLACIAN, ZERO_CROSS});
    const bool bsl = same_group(pr, {BLUR, SOBEL, LAPLACIAN});
    const bool all4 = same_group(pr, {BLUR, SOBEL, LAPLACIAN, ZERO_CROSS});
    int depth = 0;
    if (all4) depth = 4;
    else if (bsl) depth = 3;
    else if (bs && lz) depth = 2;
    else if (!same_group(pr, {BLUR, SOBEL}) && !same_group(pr, {BLUR, LAPLACIAN}) &&
             !same_group(pr, {BLUR, ZERO_CROSS}) && !same_group(pr, {LAPLACIAN, ZERO_CROSS}) &&
             !same_group(pr, {SOBEL, LAPLACIAN}) && !same_group(pr, {SOBEL, ZERO_CROSS}))
        depth = 1;
    if (!depth)
        return fail(HX_E_UNSUPPORTED,
                    "no kernel implements this fusion: fuse [blur, sobel] and [laplacian, "
                    "zero_cross], or [blur, sobel, laplacian], or all four stencils");
    // Reduction structure.
    int reduce = HX_REDUCE_SEQUENTIAL;
    if (pr.warp) reduce = HX_REDUCE_TREE;
    else if (pr.fissioned) reduce = HX_REDUCE_TWO_LEVEL;
    else if (pr.chunks)
        return fail(HX_E_UNSUPPORTED,
                    "a chunked max_gradient needs monoid-reassociate and fork-fission (or "
                    "warp-reduce) to run in parallel");
    if (reduce == HX_REDUCE_TWO_LEVEL && pr.chunks != kTreeThreads)
        return fail(HX_E_UNSUPPORTED, "the two-level max reduction is built for %d chunks",
                    kTreeThreads);
    if (depth > 1 && reduce != HX_REDUCE_TREE)
        return fail(HX_E_UNSUPPORTED,
                    "fused sweeps reduce the max with wave primitives only: apply "
                    "warp-reduce(max_gradient)");
    if (pr.pass_set && depth != 4)
        return fail(HX_E_UNSUPPORTED, "a pass structure applies to the fully fused sweep only");
    hx_schedule s{};
    s.fusion_depth = depth;
    s.reduce_mode = reduce;
    s.pass_mode = depth == 4 ? pr.pass : HX_PASS_STORE;
    // Tile: depth 1 runs every stage kernel with one tile; fused depths take
    // the sweep tile of the group holding blur.
    if (depth == 1) {
        int r = 0, c = 0;
        for (int st : {BLUR, LAPLACIAN, ZERO_CROSS, SOBEL}) {
            const int g = pr.group[st];
            if (!pr.rows[g]) continue;
            if (r && (pr.rows[g] != r || pr.cols[g] != c))
                return fail(HX_E_UNSUPPORTED,
                            "unfused stage kernels share one tile shape; got %dx%d and %dx%d",
                            r, c, pr.rows[g], pr.cols[g]);
            r = pr.rows[g];
            c = pr.cols[g];
        }
        s.tile_h = r ? r : 16;
        s.tile_w = c ? c : 64;
    } else {
        const int g = pr.group[BLUR];
        s.tile_h = pr.rows[g] ? pr.rows[g] : 64;
        s.tile_w = pr.cols[g] ? pr.cols[g] : 256;
    }
    *out = s;
    return HX_OK;
}

}  // namespace

hx_status compile_schedule(const char* text, hx_schedule* out) {
    if (!text || !out) return fail(HX_E_INVALID, "NULL argument");
    std::vector<Stmt> prog;
    hx_status st = parse(text, prog);
    if (st != HX_OK) return st;
    Program pr;
    for (int i = 0; i < NSTAGES; ++i) pr.group[i] = i;
    for (size_t i = 0; i < prog.size(); ++i) {
        st = apply(pr, prog[i], (int)i + 1);
        if (st != HX_OK) return st;
    }
    return lower(pr, out);
}

std::string schedule_text(const hx_schedule& s) {
    char buf[512];
    std::string t;
    if (s.fusion_depth == 1) {
        std::snprintf(buf, sizeof buf, "fork-tile[%d, %d](blur, laplacian, zero_cross, sobel); ",
                      s.tile_h, s.tile_w);
        t = buf;
    } else {
        if (s.fusion_depth == 2) t = "fork-fuse(blur, sobel); fork-fuse(laplacian, zero_cross); ";
        if (s.fusion_depth == 3) t = "fork-fuse(blur, sobel, laplacian); ";
        if (s.fusion_depth == 4) t = "fork-fuse(blur, sobel, laplacian, zero_cross); ";
        std::snprintf(buf, sizeof buf, "fork-tile[%d, %d](blur); ", s.tile_h, s.tile_w);
        t += buf;
    }
    if (s.reduce_mode == HX_REDUCE_TREE) t += "warp-reduce(max_gradient); ";
    if (s.reduce_mode == HX_REDUCE_TWO_LEVEL) {
        std::snprintf(buf, sizeof buf, "reduction_tree![%d](max_gradient); ", kTreeThreads);
        t += buf;
    }
    if (s.fusion_depth == 4) {
        const char* p = s.pass_mode == HX_PASS_RECOMPUTE   ? "recompute"
                        : s.pass_mode == HX_PASS_SPECULATE ? "speculate"
                                                           : "store";
        t += std::string("pass[") + p + "](threshold); ";
    }
    if (!t.empty() && t.back() == ' ') t.pop_back();
    return t;
}

}  // namespace hx

using namespace hx;

extern "C" {

hx_status hx_schedule_compile(const char* text, hx_schedule* out) {
    return compile_schedule(text, out);
}

hx_status hx_schedule_to_text(const hx_schedule* s, char* buf, size_t len) {
    if (!s || !buf || !len) return fail(HX_E_INVALID, "NULL argument");
    const std::string t = schedule_text(*s);
    if (t.size() + 1 > len) return fail(HX_E_INVALID, "buffer of %zu bytes too small", len);
    std::memcpy(buf, t.c_str(), t.size() + 1);
    return HX_OK;
}

}  // extern "C"

// Formula front end: parser, shape rule, folding and lowering to passes.
//
// Language (the DSL of Section IV-A):
//   primary := DFT(n) | I(n) | twiddle(N, M) | Permute(N, K) | ( expr )
//   expr    := primary [ op expr ]
// Both operators share one precedence level and group to the right, as in
// the grammar of Listing 2.  Kronecker product: U+2297, "(x)" or "kron";
// matrix product: U+00B7, ".", "*" or "@".  Keywords are case-insensitive
// ("identity" also names I).  A trailing vector operand after a matrix
// product (an identifier such as the input tensor of Listing 1) is accepted
// and ignored: the plan applies the formula to its input.
//
// Meaning of the factors (Eq. 2, with the readings that make it exact):
//   DFT(n)        [w_n^{j k}],  w_n = exp(-2 pi i / n)
//   I(n)          identity of size n
//   twiddle(N, M) D^N_M = diag(w_N^{i j}) at position i M + j,  i < N / M, j < M
//   Permute(N, K) Pi^N_K:  (Pi x)[i M + j] = x[j K + i],  M = N / K
// Shape rule: a Kronecker product has the product of its operands' sizes, a
// matrix product needs operands of equal size.
//
// Folding.  A product is associative, so nested products are flattened;
// sizes-1 factors, I (x) I and twiddle / Permute factors that are the
// identity (M or K equal to 1 or N) are simplified away.  Then every window
// of four factors that is Eq. 2,
//   (DFT(K) (x) I(M)) . twiddle(N, M) . (I(K) (x) DFT(M)) . Permute(N, K),
// or its transpose (DFT_N is symmetric and Pi^N_K transposed is Pi^N_M),
//   Permute(N, M) . (I(K) (x) DFT(M)) . twiddle(N, M) . (DFT(K) (x) I(M)),
// with N = K M, is replaced by DFT(N), innermost first, until none is left.
// A formula that folds to I(p) (x) DFT(n) (p >= 1) runs as p batched
// transforms of the ordinary plan for n.
//
// Lowering.  Each node acts on a vector as I_p (x) node (x) I_q:
//   A . B     -> B, then A;   A (x) B -> I_|A| (x) B, then A (x) I_|B|
//   DFT(n)    -> a codelet pass if n is a codelet radix; else, for 7-smooth
//                n, Stockham stages of the planner's radix list, or with
//                FFTC_FORMULA_EQ2 the Eq. 2 factors themselves (Permute,
//                I (x) DFT(M), twiddle, DFT(K) (x) I) recursively; n with
//                prime factors > 7 splits as n = s u (s: those factors) by
//                Eq. 2 and DFT(s) is summed directly.
#include "formula.h"

#include <ctype.h>
#include <string.h>

#include <map>
#include <memory>
#include <tuple>

namespace fftc {

namespace {

// ---- parse tree ---------------------------------------------------------------
struct Node {
    enum Kind { DFT, ID, TW, PERM, KRON, MUL } kind = DFT;
    int64_t a = 0, b = 0;
    std::unique_ptr<Node> l, r;
};

constexpr int64_t kMaxDim = int64_t(1) << 24;
constexpr int64_t kMaxDirect = 16384;
constexpr size_t kMaxPasses = 1024;
constexpr int kMaxDepth = 200;

struct Parser {
    const std::string& s;
    size_t i = 0;
    int depth = 0;
    std::string err;
    explicit Parser(const std::string& text) : s(text) {}

    void ws() {
        while (i < s.size() && isspace((unsigned char)s[i])) ++i;
    }
    bool lit(const char* t) {
        ws();
        const size_t n = strlen(t);
        if (s.compare(i, n, t) == 0) {
            i += n;
            return true;
        }
        return false;
    }
    static bool idch(char c) { return isalnum((unsigned char)c) || c == '_'; }
    bool word(const char* w) {  // case-insensitive keyword, not followed by an identifier character
        ws();
        const size_t n = strlen(w);
        if (i + n > s.size()) return false;
        for (size_t k = 0; k < n; ++k)
            if (tolower((unsigned char)s[i + k]) != tolower((unsigned char)w[k])) return false;
        if (i + n < s.size() && idch(s[i + n])) return false;
        i += n;
        return true;
    }
    bool number(int64_t* v) {
        ws();
        size_t j = i;
        while (j < s.size() && isdigit((unsigned char)s[j])) ++j;
        if (j == i || j - i > 12) return false;
        *v = std::stoll(s.substr(i, j - i));
        i = j;
        return true;
    }
    int op() {  // 1: Kronecker, 2: matrix product, 0: none
        ws();
        if (lit("\xe2\x8a\x97") || lit("(x)") || word("kron")) return 1;
        if (lit("\xc2\xb7") || lit("*") || lit("@") || lit(".")) return 2;
        return 0;
    }
    // After a matrix product: an identifier that is no keyword, followed by
    // the end of the text, is the vector operand. The word form of the
    // Kronecker product is a keyword too, so 'DFT(2) . kron' is an operator
    // with no right operand, not a product with a vector named 'kron'.
    bool trailing_operand() {
        ws();
        size_t j = i;
        if (j >= s.size() || !(isalpha((unsigned char)s[j]) || s[j] == '_')) return false;
        while (j < s.size() && idch(s[j])) ++j;
        std::string w;
        for (size_t k = i; k < j; ++k) w += (char)tolower((unsigned char)s[k]);
        if (w == "dft" || w == "i" || w == "identity" || w == "twiddle" || w == "permute" || w == "kron")
            return false;
        size_t e = j;
        while (e < s.size() && isspace((unsigned char)s[e])) ++e;
        if (e != s.size()) return false;
        i = e;
        return true;
    }
    bool args(int64_t* x, int64_t* y) {
        if (!lit("(") || !number(x)) return false;
        if (y && (!lit(",") || !number(y))) return false;
        return lit(")");
    }
    std::unique_ptr<Node> fail_at(const std::string& m) {
        if (err.empty()) err = m + " at offset " + std::to_string(i);
        return nullptr;
    }
    std::unique_ptr<Node> primary() {
        auto n = std::make_unique<Node>();
        if (word("DFT")) {
            n->kind = Node::DFT;
            if (!args(&n->a, nullptr)) return fail_at("DFT(n) expected");
        } else if (word("identity") || word("I")) {
            n->kind = Node::ID;
            if (!args(&n->a, nullptr)) return fail_at("I(n) expected");
        } else if (word("twiddle")) {
            n->kind = Node::TW;
            if (!args(&n->a, &n->b)) return fail_at("twiddle(N, M) expected");
        } else if (word("permute")) {
            n->kind = Node::PERM;
            if (!args(&n->a, &n->b)) return fail_at("Permute(N, K) expected");
        } else if (lit("(")) {
            auto e = expr();
            if (!e) return nullptr;
            if (!lit(")")) return fail_at("')' expected");
            return e;
        } else {
            return fail_at("DFT, I, twiddle, Permute or '(' expected");
        }
        return n;
    }
    std::unique_ptr<Node> expr() {
        if (++depth > kMaxDepth) return fail_at("formula nested too deeply");
        auto lhs = primary();
        std::unique_ptr<Node> res;
        if (lhs) {
            const int o = op();
            if (!o || (o == 2 && trailing_operand())) {
                res = std::move(lhs);
            } else {
                auto rhs = expr();
                if (rhs) {
                    res = std::make_unique<Node>();
                    res->kind = o == 1 ? Node::KRON : Node::MUL;
                    res->l = std::move(lhs);
                    res->r = std::move(rhs);
                }
            }
        }
        --depth;
        return res;
    }
};

// ---- canonical form: a product (left to right) of Kronecker products ------------
struct Atom;
using Factor = std::vector<Atom>;   // Kronecker product, left to right
using Expr = std::vector<Factor>;   // matrix product, left to right
struct Atom {
    enum Kind { DFT, ID, TW, PERM, SUB } kind = ID;
    int64_t a = 1, b = 1;           // DFT/ID: a = n;  TW: (N, M);  PERM: (N, K)
    std::shared_ptr<Expr> sub;      // SUB: a parenthesised product
    int64_t dim = 1;
};

Atom prim(Atom::Kind k, int64_t a, int64_t b = 0) {
    Atom t;
    t.kind = k;
    t.a = a;
    t.b = b;
    t.dim = a;
    return t;
}

int64_t factor_dim(const Factor& f) {
    int64_t d = 1;
    for (const auto& t : f) d *= t.dim;
    return d;
}

// Shape rule on the parse tree; returns the node's size or 0 with *err set.
int64_t shape(const Node* n, std::string* err) {
    switch (n->kind) {
        case Node::DFT:
        case Node::ID:
            if (n->a < 1 || n->a > kMaxDim) {
                *err = "size " + std::to_string(n->a) + " out of range [1, 2^24]";
                return 0;
            }
            return n->a;
        case Node::TW:
        case Node::PERM:
            if (n->a < 1 || n->a > kMaxDim || n->b < 1 || n->a % n->b) {
                *err = std::string(n->kind == Node::TW ? "twiddle" : "Permute") + "(" + std::to_string(n->a) +
                       ", " + std::to_string(n->b) + "): the second argument must divide the first";
                return 0;
            }
            return n->a;
        case Node::KRON: {
            const int64_t x = shape(n->l.get(), err);
            if (!x) return 0;
            const int64_t y = shape(n->r.get(), err);
            if (!y) return 0;
            if (x > kMaxDim / y) {
                *err = "Kronecker product larger than 2^24";
                return 0;
            }
            return x * y;
        }
        case Node::MUL: {
            const int64_t x = shape(n->l.get(), err);
            if (!x) return 0;
            const int64_t y = shape(n->r.get(), err);
            if (!y) return 0;
            if (x != y) {
                *err = "matrix product of operands of sizes " + std::to_string(x) + " and " + std::to_string(y);
                return 0;
            }
            return x;
        }
    }
    return 0;
}

Expr to_expr(const Node* n);

void to_atoms(const Node* n, Factor* f) {
    switch (n->kind) {
        case Node::DFT: f->push_back(prim(Atom::DFT, n->a)); break;
        case Node::ID: f->push_back(prim(Atom::ID, n->a)); break;
        case Node::TW: f->push_back(prim(Atom::TW, n->a, n->b)); break;
        case Node::PERM: f->push_back(prim(Atom::PERM, n->a, n->b)); break;
        case Node::KRON:
            to_atoms(n->l.get(), f);
            to_atoms(n->r.get(), f);
            break;
        case Node::MUL: {
            Atom t;
            t.kind = Atom::SUB;
            t.sub = std::make_shared<Expr>(to_expr(n));
            t.dim = factor_dim((*t.sub)[0]);
            f->push_back(t);
            break;
        }
    }
}

Expr to_expr(const Node* n) {
    if (n->kind == Node::MUL) {
        Expr e = to_expr(n->l.get());
        Expr r = to_expr(n->r.get());
        e.insert(e.end(), r.begin(), r.end());
        return e;
    }
    Factor f;
    to_atoms(n, &f);
    return Expr{f};
}

bool is_id(const Factor& f) { return f.size() == 1 && f[0].kind == Atom::ID; }

Factor simplify_factor(const Factor& in, bool fold);

// Simplify (and with fold, fold) a product in place.
void simplify_expr(Expr* e, bool fold) {
    for (auto& f : *e) f = simplify_factor(f, fold);
    const int64_t dim = factor_dim((*e)[0]);
    Expr kept;
    for (auto& f : *e)
        if (!is_id(f)) kept.push_back(f);
    if (kept.empty()) kept.push_back(Factor{prim(Atom::ID, dim)});
    *e = kept;
    if (!fold) return;
    auto one = [](const Factor& f, Atom::Kind k, int64_t a, int64_t b) {
        return f.size() == 1 && f[0].kind == k && f[0].a == a && (k == Atom::DFT || f[0].b == b);
    };
    auto two = [](const Factor& f, Atom::Kind k0, int64_t a0, Atom::Kind k1, int64_t a1) {
        return f.size() == 2 && f[0].kind == k0 && f[0].a == a0 && f[1].kind == k1 && f[1].a == a1;
    };
    for (bool changed = true; changed;) {
        changed = false;
        for (size_t i = 0; i + 4 <= e->size() && !changed; ++i) {
            const Factor &f0 = (*e)[i], &f1 = (*e)[i + 1], &f2 = (*e)[i + 2], &f3 = (*e)[i + 3];
            int64_t N = 0;
            // Eq. 2: (DFT_K (x) I_M) D^N_M (I_K (x) DFT_M) Pi^N_K
            if (f0.size() == 2 && f0[0].kind == Atom::DFT && f0[1].kind == Atom::ID) {
                const int64_t K = f0[0].a, M = f0[1].a;
                if (one(f1, Atom::TW, K * M, M) && two(f2, Atom::ID, K, Atom::DFT, M) &&
                    one(f3, Atom::PERM, K * M, K))
                    N = K * M;
            }
            // transpose: Pi^N_M (I_K (x) DFT_M) D^N_M (DFT_K (x) I_M)
            if (!N && f3.size() == 2 && f3[0].kind == Atom::DFT && f3[1].kind == Atom::ID) {
                const int64_t K = f3[0].a, M = f3[1].a;
                if (one(f0, Atom::PERM, K * M, M) && two(f1, Atom::ID, K, Atom::DFT, M) &&
                    one(f2, Atom::TW, K * M, M))
                    N = K * M;
            }
            if (N) {
                e->erase(e->begin() + (long)i + 1, e->begin() + (long)i + 4);
                (*e)[i] = Factor{prim(Atom::DFT, N)};
                changed = true;
            }
        }
    }
}

Factor simplify_factor(const Factor& in, bool fold) {
    Factor out;
    for (Atom t : in) {
        if (t.kind == Atom::TW && (t.b == 1 || t.b == t.a)) t = prim(Atom::ID, t.a);
        if (t.kind == Atom::PERM && (t.b == 1 || t.b == t.a)) t = prim(Atom::ID, t.a);
        if (t.kind == Atom::DFT && t.a == 1) t = prim(Atom::ID, 1);
        if (t.kind == Atom::SUB) {
            auto sub = std::make_shared<Expr>(*t.sub);
            simplify_expr(sub.get(), fold);
            if (sub->size() == 1) {  // a single Kronecker product: splice its atoms
                for (const Atom& u : (*sub)[0]) out.push_back(u);
                continue;
            }
            t.sub = sub;
        }
        out.push_back(t);
    }
    // merge neighbouring identities and drop size-1 atoms
    Factor merged;
    for (const Atom& t : out) {
        if (t.kind == Atom::ID && !merged.empty() && merged.back().kind == Atom::ID) {
            merged.back() = prim(Atom::ID, merged.back().a * t.a);
            continue;
        }
        merged.push_back(t);
    }
    Factor res;
    for (const Atom& t : merged)
        if (!(t.dim == 1 && t.kind == Atom::ID)) res.push_back(t);
    if (res.empty()) res.push_back(prim(Atom::ID, factor_dim(in)));
    return res;
}

std::string show_expr(const Expr& e);

std::string show_atom(const Atom& t) {
    switch (t.kind) {
        case Atom::DFT: return "DFT(" + std::to_string(t.a) + ")";
        case Atom::ID: return "I(" + std::to_string(t.a) + ")";
        case Atom::TW: return "twiddle(" + std::to_string(t.a) + ", " + std::to_string(t.b) + ")";
        case Atom::PERM: return "Permute(" + std::to_string(t.a) + ", " + std::to_string(t.b) + ")";
        case Atom::SUB: return "(" + show_expr(*t.sub) + ")";
    }
    return "?";
}

std::string show_expr(const Expr& e) {
    std::string s;
    for (size_t i = 0; i < e.size(); ++i) {
        if (i) s += " . ";
        const bool paren = e.size() > 1 && e[i].size() > 1;
        if (paren) s += "(";
        for (size_t j = 0; j < e[i].size(); ++j) {
            if (j) s += " (x) ";
            s += show_atom(e[i][j]);
        }
        if (paren) s += ")";
    }
    return s;
}

// ---- lowering -------------------------------------------------------------------
bool is_codelet(int64_t n) { return n == 2 || n == 3 || n == 4 || n == 5 || n == 7 || n == 8 || n == 16; }

struct Lowerer {
    FormulaProgram* prog;
    bool eq2;
    std::string err;
    std::map<std::tuple<int64_t, int64_t, int64_t, int64_t>, int64_t> table_at;

    // table of entries w_len^{a b}, a = idx / ns + a0, b = idx mod ns (shared when repeated)
    int64_t table(int64_t count, int64_t ns, int64_t len, int64_t a0) {
        const auto key = std::make_tuple(count, ns, len, a0);
        auto it = table_at.find(key);
        if (it != table_at.end()) return it->second;
        const int64_t off = prog->table_entries;
        TwSegment s;
        s.off = off;
        s.count = count;
        s.ns = ns;
        s.len = len;
        s.a0 = a0;
        prog->tables.push_back(s);
        prog->table_entries += count;
        table_at[key] = off;
        return off;
    }
    void push(const FormulaPass& ps) { prog->passes.push_back(ps); }

    void dft(int64_t n, int64_t p, int64_t q) {
        if (n == 1) return;
        FormulaPass ps;
        ps.n = n;
        ps.p = p;
        ps.q = q;
        if (is_codelet(n)) {
            ps.kind = FP_DFT;
            ps.r = (int)n;
            push(ps);
            return;
        }
        int64_t s = 1, u = n;  // u: the 7-smooth part, s: the rest
        for (int64_t f : {2, 3, 5, 7})
            while (u % f == 0) u /= f;
        s = u;
        u = n / s;
        if (s > 1 && u == 1) {
            if (n > kMaxDirect) {
                err = "DFT(" + std::to_string(n) + "): a prime factor above 7 larger than 16384 is not supported";
                return;
            }
            ps.kind = FP_DIRECT;
            ps.twoff = table(n, n, n, 1);
            push(ps);
            return;
        }
        if (s > 1) {  // Eq. 2 with K = s (summed directly), M = u
            eq2_split(n, s, p, q);
            return;
        }
        auto cands = radix_candidates(n, 1);
        if (cands.empty()) {
            err = "no factorisation for DFT(" + std::to_string(n) + ")";
            return;
        }
        const std::vector<int>& rs = cands[0];
        if (eq2) {
            eq2_split(n, rs[0], p, q);
            return;
        }
        int64_t ns = 1;
        for (int r : rs) {
            FormulaPass st;
            st.kind = FP_STAGE;
            st.n = n;
            st.r = r;
            st.ns = ns;
            st.p = p;
            st.q = q;
            if (ns > 1) st.twoff = table((r - 1) * ns, ns, ns * r, 1);
            push(st);
            ns *= r;
        }
    }
    // DFT_n = (DFT_K (x) I_M) D^n_M (I_K (x) DFT_M) Pi^n_K, applied right to left
    void eq2_split(int64_t n, int64_t K, int64_t p, int64_t q) {
        const int64_t M = n / K;
        perm(n, K, p, q);
        dft(M, p * K, q);
        diag(n, M, p, q);
        dft(K, p, M * q);
    }
    void diag(int64_t N, int64_t M, int64_t p, int64_t q) {
        if (M == 1 || M == N) return;
        FormulaPass ps;
        ps.kind = FP_DIAG;
        ps.n = N;
        ps.a = M;
        ps.p = p;
        ps.q = q;
        ps.twoff = table(N, M, N, 0);
        push(ps);
    }
    void perm(int64_t N, int64_t K, int64_t p, int64_t q) {
        if (K == 1 || K == N) return;
        FormulaPass ps;
        ps.kind = FP_PERM;
        ps.n = N;
        ps.a = K;
        ps.p = p;
        ps.q = q;
        push(ps);
    }
    void atom(const Atom& t, int64_t p, int64_t q) {
        switch (t.kind) {
            case Atom::DFT: dft(t.a, p, q); break;
            case Atom::ID: break;
            case Atom::TW: diag(t.a, t.b, p, q); break;
            case Atom::PERM: perm(t.a, t.b, p, q); break;
            case Atom::SUB: expr(*t.sub, p, q); break;
        }
    }
    void factor(const Factor& f, int64_t p, int64_t q) {
        // the operands of a Kronecker product act on separate index digits:
        // atom j is I_{p * (sizes before j)} (x) atom (x) I_{(sizes after j) * q}
        int64_t after = 1;
        for (size_t j = f.size(); j-- > 0;) {
            const int64_t before = factor_dim(f) / (after * f[j].dim);
            atom(f[j], p * before, after * q);
            after *= f[j].dim;
        }
    }
    void expr(const Expr& e, int64_t p, int64_t q) {
        for (size_t i = e.size(); i-- > 0;) factor(e[i], p, q);
    }
};

}  // namespace

fftc_status compile_formula(const std::string& text, int flags, int dtype, FormulaProgram* prog) {
    if ((flags & ~(FFTC_FORMULA_NO_FOLD | FFTC_FORMULA_EQ2 | FFTC_FORMULA_HBM_PASSES)) != 0)
        return fail(FFTC_ERR_INVALID_ARG, "formula: unknown flags");
    Parser ps(text);
    auto root = ps.expr();
    if (!root) return fail(FFTC_ERR_INVALID_ARG, "formula: " + ps.err);
    ps.ws();
    if (ps.i != text.size())
        return fail(FFTC_ERR_INVALID_ARG, "formula: unexpected text at offset " + std::to_string(ps.i));
    std::string err;
    const int64_t dim = shape(root.get(), &err);
    if (!dim) return fail(FFTC_ERR_INVALID_ARG, "formula: " + err);

    const bool fold = !(flags & FFTC_FORMULA_NO_FOLD);
    Expr e = to_expr(root.get());
    simplify_expr(&e, fold);
    *prog = FormulaProgram{};
    prog->dim = dim;
    prog->canonical = show_expr(e);
    if (fold && e.size() == 1) {
        const Factor& f = e[0];
        int64_t pp = 0, nn = 0;
        if (f.size() == 1 && f[0].kind == Atom::DFT) {
            pp = 1;
            nn = f[0].a;
        } else if (f.size() == 2 && f[0].kind == Atom::ID && f[1].kind == Atom::DFT) {
            pp = f[0].a;
            nn = f[1].a;
        }
        if (nn > 1 && is_7smooth(nn) && nn <= max_total_n(dtype)) {
            prog->folded = true;
            prog->fold_n = nn;
            prog->fold_p = pp;
            return FFTC_OK;
        }
    }
    Lowerer lw{prog, (flags & FFTC_FORMULA_EQ2) != 0, {}, {}};
    lw.expr(e, 1, 1);
    if (!lw.err.empty()) return fail(FFTC_ERR_UNSUPPORTED_SIZE, "formula: " + lw.err);
    if (prog->passes.size() > kMaxPasses)
        return fail(FFTC_ERR_UNSUPPORTED_SIZE, "formula lowers to more than 1024 passes");
    if (prog->passes.empty()) {
        FormulaPass cp;
        cp.kind = FP_COPY;
        cp.n = dim;
        prog->passes.push_back(cp);
    }
    return FFTC_OK;
}

std::string describe_formula(const FormulaProgram& prog) {
    std::string out = "dim " + std::to_string(prog.dim) + "\nformula " + prog.canonical + "\n";
    if (prog.folded) {
        out += "plan I(" + std::to_string(prog.fold_p) + ") (x) DFT(" + std::to_string(prog.fold_n) + ")\n";
        return out;
    }
    static const char* names[] = {"dft", "stage", "direct", "diag", "perm", "copy"};
    for (const auto& p : prog.passes) {
        out += names[p.kind];
        out += " n=" + std::to_string(p.n) + " p=" + std::to_string(p.p) + " q=" + std::to_string(p.q);
        if (p.kind == FP_DFT || p.kind == FP_STAGE) out += " r=" + std::to_string(p.r);
        if (p.kind == FP_STAGE) out += " ns=" + std::to_string(p.ns);
        if (p.kind == FP_DIAG) out += " M=" + std::to_string(p.a);
        if (p.kind == FP_PERM) out += " K=" + std::to_string(p.a);
        out += "\n";
    }
    return out;
}

}  // namespace fftc

// Host compiler of site-local expressions into register programs for the
// program kernel: parse, type-check, order the evaluation to use few
// registers, allocate registers.  No device code; no HIP calls.
//
// Grammar (whitespace ignored):
//   expr    := term (('+' | '-') term)*
//   term    := unary ('*' unary)*
//   unary   := '-' unary | primary
//   primary := number | 'i' | operand | func '(' expr ')' | '(' expr ')'
//   operand := 'a' .. 'h'              (operand fields 0 .. 7)
//   func    := adj | conj | transpose | trace | real | imag
// Types: real scalar, complex scalar, 3x3 complex matrix.  Scalars
// combine with matrices as multiples of the identity (s + M adds s to the
// diagonal, s * M scales), as the lattice expression templates treat a
// scalar assigned to a matrix-valued field.
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "su3_program.h"

namespace su3i {
namespace {

enum Ty { T_REAL = 0, T_COMPLEX = 1, T_MATRIX = 2 };

enum NodeKind { N_OPERAND, N_CONST, N_NEG, N_ADD, N_SUB, N_MUL, N_FUNC };
enum Func { F_ADJ, F_CONJ, F_TRANS, F_TRACE, F_REAL, F_IMAG };

struct Node {
    NodeKind kind;
    int operand = -1;
    double re = 0, im = 0;
    Func func = F_ADJ;
    std::unique_ptr<Node> l, r;
    Ty ty = T_REAL;
    int need = 0;  // registers to evaluate (operands are preloaded)
};

struct Parser {
    const char *p;
    std::string err;

    void skip()
    {
        while (*p && std::isspace((unsigned char)*p))
            ++p;
    }
    bool fail(const std::string &m)
    {
        if (err.empty())
            err = m;
        return false;
    }

    std::unique_ptr<Node> expr()
    {
        auto n = term();
        for (;;) {
            skip();
            if (!n || (*p != '+' && *p != '-'))
                return n;
            const char op = *p++;
            auto r = term();
            if (!r)
                return nullptr;
            auto m = std::make_unique<Node>();
            m->kind = op == '+' ? N_ADD : N_SUB;
            m->l = std::move(n);
            m->r = std::move(r);
            n = std::move(m);
        }
    }

    std::unique_ptr<Node> term()
    {
        auto n = unary();
        for (;;) {
            skip();
            if (!n || *p != '*')
                return n;
            ++p;
            auto r = unary();
            if (!r)
                return nullptr;
            auto m = std::make_unique<Node>();
            m->kind = N_MUL;
            m->l = std::move(n);
            m->r = std::move(r);
            n = std::move(m);
        }
    }

    std::unique_ptr<Node> unary()
    {
        skip();
        if (*p == '-') {
            ++p;
            auto c = unary();
            if (!c)
                return nullptr;
            auto m = std::make_unique<Node>();
            m->kind = N_NEG;
            m->l = std::move(c);
            return m;
        }
        return primary();
    }

    std::unique_ptr<Node> primary()
    {
        skip();
        if (std::isdigit((unsigned char)*p) || *p == '.') {
            char *end = nullptr;
            const double v = std::strtod(p, &end);
            if (end == p) {
                fail("malformed number");
                return nullptr;
            }
            p = end;
            auto m = std::make_unique<Node>();
            m->kind = N_CONST;
            m->re = v;
            return m;
        }
        if (*p == '(') {
            ++p;
            auto n = expr();
            skip();
            if (!n)
                return nullptr;
            if (*p != ')') {
                fail("expected ')'");
                return nullptr;
            }
            ++p;
            return n;
        }
        if (std::isalpha((unsigned char)*p)) {
            const char *b = p;
            while (std::isalnum((unsigned char)*p) || *p == '_')
                ++p;
            const std::string id(b, p);
            if (id.size() == 1 && id[0] >= 'a' && id[0] <= 'h') {
                auto m = std::make_unique<Node>();
                m->kind = N_OPERAND;
                m->operand = id[0] - 'a';
                return m;
            }
            if (id == "i") {
                auto m = std::make_unique<Node>();
                m->kind = N_CONST;
                m->im = 1.0;
                return m;
            }
            static const struct {
                const char *name;
                Func f;
            } funcs[] = {{"adj", F_ADJ},     {"conj", F_CONJ}, {"transpose", F_TRANS},
                         {"trace", F_TRACE}, {"real", F_REAL}, {"imag", F_IMAG}};
            for (const auto &fn : funcs)
                if (id == fn.name) {
                    skip();
                    if (*p != '(') {
                        fail("expected '(' after " + id);
                        return nullptr;
                    }
                    ++p;
                    auto c = expr();
                    skip();
                    if (!c)
                        return nullptr;
                    if (*p != ')') {
                        fail("expected ')'");
                        return nullptr;
                    }
                    ++p;
                    auto m = std::make_unique<Node>();
                    m->kind = N_FUNC;
                    m->func = fn.f;
                    m->l = std::move(c);
                    return m;
                }
            fail("unknown name '" + id + "' (operands are a..h)");
            return nullptr;
        }
        fail(*p ? std::string("unexpected '") + *p + "'" : "unexpected end");
        return nullptr;
    }
};

// Types, SU(3)-closure and register needs (Sethi-Ullman numbers).
bool annotate(Node *n, int nops, const int *kinds, bool *closed, std::string *err)
{
    switch (n->kind) {
    case N_OPERAND:
        if (n->operand >= nops) {
            *err = "operand '" + std::string(1, char('a' + n->operand)) +
                   "' beyond the operand count";
            return false;
        }
        switch (kinds[n->operand]) {
        case FK_MATRIX: n->ty = T_MATRIX; break;
        case FK_REAL: n->ty = T_REAL; break;
        case FK_COMPLEX: n->ty = T_COMPLEX; break;
        default: *err = "spinor operands are not supported in expressions"; return false;
        }
        n->need = 0;
        return true;
    case N_CONST:
        n->ty = n->im != 0.0 ? T_COMPLEX : T_REAL;
        n->need = 1;
        *closed = false;
        return true;
    case N_NEG:
        if (!annotate(n->l.get(), nops, kinds, closed, err))
            return false;
        n->ty = n->l->ty;
        n->need = n->l->need > 1 ? n->l->need : 1;
        *closed = false;
        return true;
    case N_FUNC: {
        if (!annotate(n->l.get(), nops, kinds, closed, err))
            return false;
        const Ty c = n->l->ty;
        switch (n->func) {
        case F_ADJ:
        case F_CONJ:
        case F_TRANS: n->ty = c; break;
        case F_TRACE:
            n->ty = c == T_MATRIX ? T_COMPLEX : c;
            *closed = false;
            break;
        case F_REAL:
        case F_IMAG:
            if (c == T_MATRIX) {
                *err = "real() and imag() take scalars";
                return false;
            }
            n->ty = T_REAL;
            *closed = false;
            break;
        }
        n->need = n->l->need > 1 ? n->l->need : 1;
        return true;
    }
    default: {
        if (!annotate(n->l.get(), nops, kinds, closed, err) ||
            !annotate(n->r.get(), nops, kinds, closed, err))
            return false;
        const Ty a = n->l->ty, b = n->r->ty;
        if (a == T_MATRIX || b == T_MATRIX)
            n->ty = T_MATRIX;
        else
            n->ty = (a == T_COMPLEX || b == T_COMPLEX) ? T_COMPLEX : T_REAL;
        if (!(n->kind == N_MUL && a == T_MATRIX && b == T_MATRIX))
            *closed = false;
        const int l = n->l->need, r = n->r->need;
        n->need = l == r ? l + 1 : (l > r ? l : r);
        if (n->need < 1)
            n->need = 1;
        return true;
    }
    }
}

// Code generation over virtual registers: operand k is vreg k; every
// other value gets a fresh vreg.
struct Gen {
    std::vector<ProgInstr> ins;  // operands in virtual registers
    std::vector<std::pair<double, double>> imm;
    int nvreg;
    std::string err;

    int fresh() { return nvreg++; }

    int emit(uint8_t op, int a, int b)
    {
        const int d = fresh();
        ins.push_back(ProgInstr{op, (uint8_t)d, (uint8_t)a, (uint8_t)b});
        return d;
    }

    int gen(const Node *n)
    {
        switch (n->kind) {
        case N_OPERAND: return n->operand;
        case N_CONST: {
            if ((int)imm.size() >= kProgMaxImm) {
                err = "too many constants";
                return -1;
            }
            imm.push_back({n->re, n->im});
            return emit(OP_CONST, (int)imm.size() - 1, 0);
        }
        case N_NEG: {
            const int a = gen(n->l.get());
            if (a < 0)
                return -1;
            return emit(n->ty == T_MATRIX ? OP_NEG_M : OP_NEG_S, a, a);
        }
        case N_FUNC: {
            const int a = gen(n->l.get());
            if (a < 0)
                return -1;
            const Ty c = n->l->ty;
            switch (n->func) {
            case F_ADJ:
                if (c == T_MATRIX)
                    return emit(OP_ADJ_M, a, a);
                return c == T_COMPLEX ? emit(OP_CONJ_S, a, a) : a;
            case F_CONJ:
                if (c == T_MATRIX)
                    return emit(OP_CONJ_M, a, a);
                return c == T_COMPLEX ? emit(OP_CONJ_S, a, a) : a;
            case F_TRANS: return c == T_MATRIX ? emit(OP_TRANS_M, a, a) : a;
            case F_TRACE: return c == T_MATRIX ? emit(OP_TRACE, a, a) : a;
            case F_REAL: return c == T_COMPLEX ? emit(OP_REAL, a, a) : a;
            case F_IMAG: return emit(OP_IMAG, a, a);
            }
            return -1;
        }
        default: {
            // the operand needing more registers first (Sethi-Ullman)
            int a, b;
            if (n->r->need > n->l->need) {
                b = gen(n->r.get());
                a = b < 0 ? -1 : gen(n->l.get());
            } else {
                a = gen(n->l.get());
                b = a < 0 ? -1 : gen(n->r.get());
            }
            if (a < 0 || b < 0)
                return -1;
            const bool ma = n->l->ty == T_MATRIX, mb = n->r->ty == T_MATRIX;
            uint8_t op;
            if (n->kind == N_MUL)
                op = ma ? (mb ? OP_MUL_MM : OP_MUL_MS) : (mb ? OP_MUL_SM : OP_MUL_SS);
            else if (n->kind == N_ADD)
                op = ma ? (mb ? OP_ADD_MM : OP_ADD_MS) : (mb ? OP_ADD_SM : OP_ADD_SS);
            else
                op = ma ? (mb ? OP_SUB_MM : OP_SUB_MS) : (mb ? OP_SUB_SM : OP_SUB_SS);
            return emit(op, a, b);
        }
        }
    }
};

}  // namespace

bool compile_program(const char *text, int nops, const int *kinds,
                     ProgCode *out, char *errbuf, size_t errlen)
{
    auto failmsg = [&](const std::string &m) {
        if (errbuf && errlen)
            std::snprintf(errbuf, errlen, "%s", m.c_str());
        return false;
    };
    if (!text)
        return failmsg("expression is NULL");
    if (nops < 0 || nops > kProgMaxOps)
        return failmsg("at most 8 operands");
    Parser ps{text, {}};
    std::unique_ptr<Node> root = ps.expr();
    ps.skip();
    if (!root)
        return failmsg("parse error: " + ps.err);
    if (*ps.p)
        return failmsg(std::string("parse error: unexpected '") + *ps.p + "'");
    bool closed = true;
    std::string err;
    if (!annotate(root.get(), nops, kinds, &closed, &err))
        return failmsg(err);

    Gen g;
    g.nvreg = nops;
    int res = g.gen(root.get());
    if (res < 0)
        return failmsg(g.err);
    if ((int)g.ins.size() > kProgMaxInstr)
        return failmsg("expression too long");

    // Linear-scan allocation of physical registers: operand k starts in
    // register k; a register is free after the last read of its value
    // (the result stays live to the end).
    const int nv = g.nvreg;
    std::vector<int> last(nv, -1), phys(nv, -1);
    for (int t = 0; t < (int)g.ins.size(); ++t) {
        if (g.ins[t].op == OP_CONST)
            continue;  // its `a` is a constant index
        last[g.ins[t].a] = t;
        last[g.ins[t].b] = t;
    }
    last[res] = (int)g.ins.size();
    std::vector<int> owner(kProgMaxRegs, -1);  // vreg held by each register
    for (int k = 0; k < nops; ++k) {
        phys[k] = k;
        owner[k] = last[k] >= 0 ? k : -1;  // unused operands free at once
    }
    int maxreg = nops;
    for (int t = 0; t < (int)g.ins.size(); ++t) {
        ProgInstr &in = g.ins[t];
        const bool is_const = in.op == OP_CONST;
        const int va = in.a, vb = in.b, vd = in.d;
        // free the inputs read for the last time here (the output may
        // reuse their register: instructions read before they write)
        if (!is_const) {
            for (int v : {va, vb})
                if (last[v] == t && owner[phys[v]] == v)
                    owner[phys[v]] = -1;
        }
        int r = -1;
        for (int k = 0; k < kProgMaxRegs; ++k)
            if (owner[k] < 0) {
                r = k;
                break;
            }
        if (r < 0)
            return failmsg("expression needs more than 8 registers");
        owner[r] = vd;
        phys[vd] = r;
        if (r + 1 > maxreg)
            maxreg = r + 1;
        in.d = (uint8_t)r;
        if (!is_const) {
            in.a = (uint8_t)phys[va];
            in.b = (uint8_t)phys[vb];
        }
    }

    std::memset(out, 0, sizeof *out);
    for (size_t t = 0; t < g.ins.size(); ++t)
        out->ins[t] = g.ins[t];
    out->ninstr = (int)g.ins.size();
    for (size_t k = 0; k < g.imm.size(); ++k) {
        out->imm[k][0] = g.imm[k].first;
        out->imm[k][1] = g.imm[k].second;
    }
    out->nimm = (int)g.imm.size();
    out->result = phys[res];
    out->result_kind = root->ty == T_MATRIX ? FK_MATRIX
                       : root->ty == T_COMPLEX ? FK_COMPLEX
                                               : FK_REAL;
    out->nregs = maxreg < 1 ? 1 : maxreg;
    out->nops = nops;
    out->su3_closed = closed && root->ty == T_MATRIX;
    struct Walk {
        static bool any_matrix(const Node *n)
        {
            return n && (n->ty == T_MATRIX || any_matrix(n->l.get()) ||
                         any_matrix(n->r.get()));
        }
        static bool all_real(const Node *n)
        {
            return !n || (n->ty == T_REAL && all_real(n->l.get()) &&
                          all_real(n->r.get()));
        }
    };
    out->scalar_only = !Walk::any_matrix(root.get());
    out->real_only = Walk::all_real(root.get());
    out->used = 0;
    for (int k = 0; k < nops; ++k)
        if (last[k] >= 0)
            out->used |= 1u << k;
    return true;
}

}  // namespace su3i

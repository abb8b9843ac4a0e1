// Reader of the Bayesian Interchange Format (BIF), the text format in which
// the public benchmark networks of the paper's evaluation (Section 3) are
// distributed.  It yields the same host network as the library's own .fbn
// text: variables numbered in declaration order, each CPT laid out with the
// parents in the order the probability block lists them and the variable
// itself fastest.
//
// Accepted grammar (whitespace-insensitive; // and /* */ comments):
//   network NAME { property ... ; ... }
//   variable NAME { type discrete [ R ] { STATE, STATE, ... } ; property ... ; }
//   probability ( NAME ) { table P, P, ... ; }
//   probability ( NAME | PARENT, PARENT, ... ) {
//       ( STATE, STATE, ... ) P, P, ... ;    one row per parent assignment
//       default P, P, ... ;                   rows not listed otherwise
//   }
// Names and states are words of letters, digits and the characters
// _ - . + ' (double quotes around a word are dropped).  A conditional
// distribution given as one flat `table` is refused: the published
// descriptions of its entry order disagree, so it is ambiguous.  A row whose
// probabilities sum to within 1e-3 of one is divided by its sum (published
// files print rounded decimals); a larger deviation is an error.
#include <cerrno>
#include <cmath>
#include <cstdlib>
#include <map>
#include <string>
#include <vector>

#include "fbn_internal.h"

namespace fbn {
namespace {

struct Tok {
    std::string s;
    bool punct;
    int line;
};

bool is_punct(char ch) {
    return ch == '{' || ch == '}' || ch == '(' || ch == ')' || ch == '[' || ch == ']' || ch == ',' || ch == ';' ||
           ch == '|';
}

bool is_space(char ch) { return ch == ' ' || ch == '\t' || ch == '\n' || ch == '\r' || ch == '\f' || ch == '\v'; }

std::string tokenize(const char* p, size_t len, std::vector<Tok>& out) {
    const char* end = p + len;
    int line = 1;
    while (p < end) {
        const char ch = *p;
        if (ch == '\n') {
            line++;
            p++;
        } else if (is_space(ch)) {
            p++;
        } else if (ch == '/' && p + 1 < end && p[1] == '/') {
            while (p < end && *p != '\n') p++;
        } else if (ch == '/' && p + 1 < end && p[1] == '*') {
            p += 2;
            while (p + 1 < end && !(p[0] == '*' && p[1] == '/')) {
                if (*p == '\n') line++;
                p++;
            }
            if (p + 1 >= end) return "unterminated comment";
            p += 2;
        } else if (is_punct(ch)) {
            out.push_back({std::string(1, ch), true, line});
            p++;
        } else if (ch == '"') {
            const char* s = ++p;
            while (p < end && *p != '"') {
                if (*p == '\n') line++;
                p++;
            }
            if (p >= end) return "unterminated quoted name";
            out.push_back({std::string(s, (size_t)(p - s)), false, line});
            p++;
        } else {
            const char* s = p;
            while (p < end && !is_space(*p) && !is_punct(*p) && *p != '"' &&
                   !(*p == '/' && p + 1 < end && (p[1] == '/' || p[1] == '*')))
                p++;
            out.push_back({std::string(s, (size_t)(p - s)), false, line});
        }
    }
    return "";
}

struct Parser {
    std::vector<Tok> t;
    size_t k = 0;
    std::string err;

    bool fail(const std::string& m) {
        if (err.empty()) err = "line " + std::to_string(k < t.size() ? t[k].line : (t.empty() ? 0 : t.back().line)) +
                               ": " + m;
        return false;
    }
    bool at_end() const { return k >= t.size(); }
    bool peek(const char* s) const { return k < t.size() && t[k].s == s; }
    bool expect(const char* s) {
        if (!peek(s)) return fail(std::string("expected '") + s + "'");
        k++;
        return true;
    }
    bool word(std::string& w) {
        if (at_end() || t[k].punct) return fail("expected a name");
        w = t[k++].s;
        return true;
    }
    bool number(double& x) {
        std::string w;
        if (!word(w)) return false;
        char* e = nullptr;
        errno = 0;
        x = std::strtod(w.c_str(), &e);
        if (errno || !e || *e) {
            k--;
            return fail("bad number '" + w + "'");
        }
        return true;
    }
    // skip a balanced { ... } block (properties and the network block)
    bool skip_block() {
        if (!expect("{")) return false;
        int depth = 1;
        while (!at_end() && depth > 0) {
            if (t[k].punct && t[k].s == "{") depth++;
            if (t[k].punct && t[k].s == "}") depth--;
            k++;
        }
        return depth == 0 || fail("unbalanced braces");
    }
    // skip "property ... ;"
    bool skip_property() {
        while (!at_end() && !(t[k].punct && t[k].s == ";")) k++;
        return expect(";");
    }
    // comma-separated list of words or numbers up to (not including) `close`
    bool list(std::vector<std::string>& out, const char* close) {
        out.clear();
        while (!peek(close)) {
            std::string w;
            if (!word(w)) return false;
            out.push_back(w);
            if (peek(",")) k++;
            else if (!peek(close)) return fail(std::string("expected ',' or '") + close + "'");
        }
        return true;
    }
    bool numbers(std::vector<double>& out) {
        out.clear();
        while (!peek(";")) {
            double x;
            if (!number(x)) return false;
            out.push_back(x);
            if (peek(",")) k++;
        }
        k++;
        return true;
    }
};

}  // namespace

std::string parse_bif(const char* text, size_t len, Net& net, std::vector<std::string>& names,
                      std::vector<std::vector<std::string>>& states) {
    Parser P;
    std::string e = tokenize(text, len, P.t);
    if (!e.empty()) return e;
    std::map<std::string, int> id;
    names.clear();
    states.clear();
    struct Prob {
        int v;
        std::vector<int> parents;
        size_t tok;
    };
    std::vector<Prob> probs;
    // pass 1: variables (declarations may follow the probability blocks)
    while (!P.at_end()) {
        std::string kw;
        if (!P.word(kw)) return P.err;
        if (kw == "network") {
            std::string nm;
            if (!P.word(nm) || !P.skip_block()) return P.err;
        } else if (kw == "variable") {
            std::string nm;
            if (!P.word(nm) || !P.expect("{")) return P.err;
            if (id.count(nm)) return (P.fail("variable '" + nm + "' declared twice"), P.err);
            std::vector<std::string> st;
            long long r = -1;
            while (!P.peek("}")) {
                std::string w;
                if (!P.word(w)) return P.err;
                if (w == "property") {
                    if (!P.skip_property()) return P.err;
                } else if (w == "type") {
                    std::string d, rs;
                    if (!P.word(d) || d != "discrete") return (P.fail("only discrete variables"), P.err);
                    if (!P.expect("[") || !P.word(rs) || !P.expect("]") || !P.expect("{")) return P.err;
                    char* end = nullptr;
                    r = std::strtoll(rs.c_str(), &end, 10);
                    if (!end || *end || r < 2) return (P.fail("bad state count '" + rs + "'"), P.err);
                    if (!P.list(st, "}") || !P.expect("}") || !P.expect(";")) return P.err;
                    if ((long long)st.size() != r) return (P.fail("state count differs from the list"), P.err);
                    for (size_t a = 0; a < st.size(); a++)
                        for (size_t b = 0; b < a; b++)
                            if (st[a] == st[b]) return (P.fail("state '" + st[a] + "' repeated"), P.err);
                } else {
                    return (P.fail("unknown variable field '" + w + "'"), P.err);
                }
            }
            P.k++;
            if (r < 0) return (P.fail("variable '" + nm + "' has no type"), P.err);
            id[nm] = (int)names.size();
            names.push_back(nm);
            states.push_back(st);
        } else if (kw == "probability") {
            // skipped in this pass
            if (!P.expect("(")) return P.err;
            while (!P.at_end() && !P.peek(")")) P.k++;
            if (!P.expect(")") || !P.skip_block()) return P.err;
        } else {
            return (P.fail("unknown block '" + kw + "'"), P.err);
        }
    }
    const int n = (int)names.size();
    if (n == 0) return "no variables";
    net.n = n;
    net.card.assign((size_t)n, 0);
    net.parents.assign((size_t)n, {});
    net.cpt.assign((size_t)n, {});
    for (int v = 0; v < n; v++) net.card[(size_t)v] = (int)states[(size_t)v].size();
    std::vector<char> has((size_t)n, 0);
    // pass 2: probability blocks
    P.k = 0;
    while (!P.at_end()) {
        std::string kw;
        P.word(kw);
        if (kw != "probability") {
            std::string nm;
            P.word(nm);
            P.skip_block();
            continue;
        }
        if (!P.expect("(")) return P.err;
        std::string child;
        if (!P.word(child)) return P.err;
        if (!id.count(child)) return (P.fail("probability of undeclared variable '" + child + "'"), P.err);
        const int v = id[child];
        if (has[(size_t)v]) return (P.fail("second probability block for '" + child + "'"), P.err);
        has[(size_t)v] = 1;
        std::vector<std::string> pn;
        if (P.peek("|")) {
            P.k++;
            if (!P.list(pn, ")")) return P.err;
        }
        if (!P.expect(")") || !P.expect("{")) return P.err;
        std::vector<int>& par = net.parents[(size_t)v];
        for (const auto& p : pn) {
            if (!id.count(p)) return (P.fail("undeclared parent '" + p + "'"), P.err);
            par.push_back(id[p]);
        }
        const uint64_t r = (uint64_t)net.card[(size_t)v];
        uint64_t rows = 1;
        for (int p : par) {
            rows *= (uint64_t)net.card[(size_t)p];
            if (rows > (1ull << 31)) return (P.fail("CPT of '" + child + "' too large"), P.err);
        }
        std::vector<double>& cpt = net.cpt[(size_t)v];
        cpt.assign(rows * r, 0.0);
        std::vector<char> got(rows, 0);
        std::vector<double> def;
        while (!P.peek("}")) {
            if (P.at_end()) return (P.fail("unterminated probability block"), P.err);
            if (P.peek("(")) {
                P.k++;
                std::vector<std::string> ps;
                if (!P.list(ps, ")") || !P.expect(")")) return P.err;
                if (ps.size() != par.size()) return (P.fail("row names " + std::to_string(ps.size()) +
                                                            " parent states, expected " + std::to_string(par.size())),
                                                     P.err);
                uint64_t row = 0;
                for (size_t a = 0; a < ps.size(); a++) {
                    const auto& sl = states[(size_t)par[a]];
                    size_t x = 0;
                    while (x < sl.size() && sl[x] != ps[a]) x++;
                    if (x == sl.size()) return (P.fail("unknown state '" + ps[a] + "' of '" + pn[a] + "'"), P.err);
                    row = row * (uint64_t)sl.size() + (uint64_t)x;
                }
                std::vector<double> vals;
                if (!P.numbers(vals)) return P.err;
                if (vals.size() != r) return (P.fail("row of '" + child + "' has " + std::to_string(vals.size()) +
                                                     " entries, expected " + std::to_string(r)), P.err);
                if (got[row]) return (P.fail("row of '" + child + "' given twice"), P.err);
                got[row] = 1;
                for (uint64_t x = 0; x < r; x++) cpt[row * r + x] = vals[x];
            } else {
                std::string w;
                if (!P.word(w)) return P.err;
                if (w == "property") {
                    if (!P.skip_property()) return P.err;
                } else if (w == "default") {
                    if (!P.numbers(def)) return P.err;
                    if (def.size() != r) return (P.fail("default row of '" + child + "' has the wrong length"), P.err);
                } else if (w == "table") {
                    if (!par.empty())
                        return (P.fail("a flat table for the conditional distribution of '" + child +
                                       "' is ambiguous; give one row per parent assignment"), P.err);
                    std::vector<double> vals;
                    if (!P.numbers(vals)) return P.err;
                    if (vals.size() != r) return (P.fail("table of '" + child + "' has the wrong length"), P.err);
                    for (uint64_t x = 0; x < r; x++) cpt[x] = vals[x];
                    got[0] = 1;
                } else {
                    return (P.fail("unknown entry '" + w + "' in the probability of '" + child + "'"), P.err);
                }
            }
        }
        P.k++;
        for (uint64_t row = 0; row < rows; row++) {
            if (got[row]) continue;
            if (def.empty()) return "variable '" + child + "': no probabilities for parent assignment " +
                                    std::to_string(row);
            for (uint64_t x = 0; x < r; x++) cpt[row * r + x] = def[x];
        }
        // rows printed as rounded decimals: renormalise small deviations
        for (uint64_t row = 0; row < rows; row++) {
            double s = 0.0;
            for (uint64_t x = 0; x < r; x++) {
                const double p = cpt[row * r + x];
                if (!std::isfinite(p) || p < 0.0) return "variable '" + child + "': probability not finite and >= 0";
                s += p;
            }
            if (std::fabs(s - 1.0) > 1e-3) return "variable '" + child + "': a row sums to " + std::to_string(s);
            if (std::fabs(s - 1.0) > 1e-12)
                for (uint64_t x = 0; x < r; x++) cpt[row * r + x] /= s;
        }
    }
    for (int v = 0; v < n; v++)
        if (!has[(size_t)v]) return "variable '" + names[(size_t)v] + "' has no probability block";
    return "";
}

}  // namespace fbn

// Query compilation: query string -> epsilon-free NFA table (rpq_nfa).
//
// The automaton is the Glushkov position automaton: state 0 is the initial
// state and state p >= 1 is the p-th label occurrence from the left.  From
// the nullable / first / last / follow sets of the expression:
//   delta(0, l) = first positions labelled l,
//   delta(p, l) = positions in follow(p) labelled l,
//   final       = last positions, plus state 0 when the empty word matches.
// It has one state per label occurrence plus one (4 states for a.b.c*), no
// epsilon moves, and every transition into a state carries that state's
// label, which is what the traversal kernels exploit (Section 2.2, the
// automata plan of Figure 2(a)).
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rpq.h"

namespace rpq {
void set_error(const char* fmt, ...);
void clear_error();
const char* last_error_cstr();
}  // namespace rpq

namespace {

struct Node {
    enum Kind { LAB, CAT, ALT, STAR, PLUS, OPT } kind;
    int a = -1, b = -1;   // children
    int pos = 0;          // position id (LAB)
};

struct Parser {
    const char* s;
    size_t i = 0, n;
    const char* const* names;
    uint32_t n_labels;
    std::vector<Node> nodes;
    std::vector<uint32_t> pos_label{0};   // pos_label[p] for p >= 1
    std::string err;

    void ws() {
        while (i < n && (s[i] == ' ' || s[i] == '\t' || s[i] == '\n' || s[i] == '\r')) ++i;
    }
    bool is_dot() {
        if (i < n && s[i] == '.') return true;
        return i + 1 < n && (unsigned char)s[i] == 0xC2 && (unsigned char)s[i + 1] == 0xB7;   // U+00B7
    }
    void skip_dot() { i += (s[i] == '.') ? 1 : 2; }
    // longest label name matching at i, or -1
    int match_label(size_t* len) {
        int best = -1;
        size_t bl = 0;
        for (uint32_t l = 0; l < n_labels; ++l) {
            const size_t k = std::strlen(names[l]);
            if (k == 0 || k <= bl || i + k > n) continue;
            if (std::memcmp(s + i, names[l], k) == 0) {
                best = (int)l;
                bl = k;
            }
        }
        *len = bl;
        return best;
    }
    bool starts_atom() {
        ws();
        if (i >= n) return false;
        if (s[i] == '(') return true;
        size_t k;
        return match_label(&k) >= 0;
    }
    int add(Node nd) {
        nodes.push_back(nd);
        return (int)nodes.size() - 1;
    }
    int alt() {
        int x = cat();
        if (x < 0) return -1;
        for (;;) {
            ws();
            if (i < n && s[i] == '|') {
                ++i;
                int y = cat();
                if (y < 0) return -1;
                x = add(Node{Node::ALT, x, y, 0});
            } else {
                return x;
            }
        }
    }
    int cat() {
        int x = post();
        if (x < 0) return -1;
        for (;;) {
            ws();
            if (i < n && is_dot()) {
                skip_dot();
                int y = post();
                if (y < 0) return -1;
                x = add(Node{Node::CAT, x, y, 0});
            } else if (starts_atom()) {
                int y = post();
                if (y < 0) return -1;
                x = add(Node{Node::CAT, x, y, 0});
            } else {
                return x;
            }
        }
    }
    int post() {
        int x = atom();
        if (x < 0) return -1;
        for (;;) {
            ws();
            if (i < n && (s[i] == '*' || s[i] == '+' || s[i] == '?')) {
                const char c = s[i++];
                x = add(Node{c == '*' ? Node::STAR : c == '+' ? Node::PLUS : Node::OPT, x, -1, 0});
            } else {
                return x;
            }
        }
    }
    int atom() {
        ws();
        if (i >= n) {
            err = "unexpected end of query";
            return -1;
        }
        if (s[i] == '(') {
            ++i;
            int x = alt();
            if (x < 0) return -1;
            ws();
            if (i >= n || s[i] != ')') {
                err = "missing ')'";
                return -1;
            }
            ++i;
            return x;
        }
        size_t k;
        const int l = match_label(&k);
        if (l < 0) {
            err = std::string("unknown label at '") + (s + i) + "'";
            return -1;
        }
        i += k;
        pos_label.push_back((uint32_t)l);
        Node nd{Node::LAB, -1, -1, (int)pos_label.size() - 1};
        return add(nd);
    }
};

struct Sets {
    bool nullable;
    uint32_t first, last;   // bitmasks over positions (bit p)
};

Sets glushkov_sets(const std::vector<Node>& nodes, int x, std::vector<uint32_t>& follow) {
    const Node& nd = nodes[x];
    switch (nd.kind) {
        case Node::LAB: {
            const uint32_t m = 1u << nd.pos;
            return Sets{false, m, m};
        }
        case Node::CAT: {
            const Sets A = glushkov_sets(nodes, nd.a, follow);
            const Sets B = glushkov_sets(nodes, nd.b, follow);
            for (int p = 1; p < 32; ++p)
                if (A.last >> p & 1) follow[p] |= B.first;
            return Sets{A.nullable && B.nullable, A.nullable ? (A.first | B.first) : A.first,
                        B.nullable ? (A.last | B.last) : B.last};
        }
        case Node::ALT: {
            const Sets A = glushkov_sets(nodes, nd.a, follow);
            const Sets B = glushkov_sets(nodes, nd.b, follow);
            return Sets{A.nullable || B.nullable, A.first | B.first, A.last | B.last};
        }
        case Node::STAR:
        case Node::PLUS: {
            const Sets A = glushkov_sets(nodes, nd.a, follow);
            for (int p = 1; p < 32; ++p)
                if (A.last >> p & 1) follow[p] |= A.first;
            return Sets{nd.kind == Node::STAR ? true : A.nullable, A.first, A.last};
        }
        case Node::OPT: {
            const Sets A = glushkov_sets(nodes, nd.a, follow);
            return Sets{true, A.first, A.last};
        }
    }
    return Sets{false, 0, 0};
}

}  // namespace

extern "C" {

const char* rpq_last_error(void) { return rpq::last_error_cstr(); }

int rpq_abi_version(void) { return RPQ_ABI_VERSION; }

int rpq_nfa_compile(const char* regex, const char* const* label_names, uint32_t n_labels, rpq_nfa* out) {
    rpq::clear_error();
    if (!regex || !label_names || !out || n_labels == 0 || n_labels > RPQ_MAX_LABELS) {
        rpq::set_error("invalid arguments to rpq_nfa_compile");
        return RPQ_EINVAL;
    }
    for (uint32_t l = 0; l < n_labels; ++l)
        if (!label_names[l]) {
            rpq::set_error("label name %u is NULL", l);
            return RPQ_EINVAL;
        }
    Parser P{regex, 0, std::strlen(regex), label_names, n_labels, {}, {0}, {}};
    P.ws();
    if (P.i >= P.n) {
        rpq::set_error("empty query");
        return RPQ_EINVAL;
    }
    // count label occurrences first so that over-long queries fail cleanly
    const int root = P.alt();
    if (root < 0) {
        rpq::set_error("query syntax error: %s", P.err.c_str());
        return RPQ_EINVAL;
    }
    P.ws();
    if (P.i != P.n) {
        rpq::set_error("query syntax error: trailing input at '%s'", regex + P.i);
        return RPQ_EINVAL;
    }
    const uint32_t n_pos = (uint32_t)P.pos_label.size() - 1;
    if (n_pos + 1 > RPQ_MAX_STATES) {
        rpq::set_error("query has %u label occurrences; at most %d are supported", n_pos, RPQ_MAX_STATES - 1);
        return RPQ_EUNSUPPORTED;
    }
    std::vector<uint32_t> follow(32, 0);
    const Sets S = glushkov_sets(P.nodes, root, follow);
    std::memset(out, 0, sizeof *out);
    out->n_states = n_pos + 1;
    out->n_labels = n_labels;
    out->initial_mask = 1u;
    out->final_mask = S.last | (S.nullable ? 1u : 0u);
    uint32_t with_label[RPQ_MAX_LABELS] = {};
    for (uint32_t p = 1; p <= n_pos; ++p) with_label[P.pos_label[p]] |= 1u << p;
    for (uint32_t l = 0; l < n_labels; ++l) {
        out->delta[0 * RPQ_MAX_LABELS + l] = S.first & with_label[l];
        for (uint32_t p = 1; p <= n_pos; ++p) out->delta[p * RPQ_MAX_LABELS + l] = follow[p] & with_label[l];
    }
    return RPQ_OK;
}

int rpq_nfa_reverse(const rpq_nfa* in, rpq_nfa* out) {
    rpq::clear_error();
    if (!in || !out || in->n_states == 0 || in->n_states > RPQ_MAX_STATES || in->n_labels == 0 ||
        in->n_labels > RPQ_MAX_LABELS) {
        rpq::set_error("invalid automaton");
        return RPQ_EINVAL;
    }
    rpq_nfa r;
    std::memset(&r, 0, sizeof r);
    r.n_states = in->n_states;
    r.n_labels = in->n_labels;
    r.initial_mask = in->final_mask;
    r.final_mask = in->initial_mask;
    for (uint32_t q = 0; q < in->n_states; ++q)
        for (uint32_t l = 0; l < in->n_labels; ++l) {
            uint32_t m = in->delta[q * RPQ_MAX_LABELS + l];
            while (m) {
                const int p = __builtin_ctz(m);
                m &= m - 1;
                r.delta[p * RPQ_MAX_LABELS + l] |= 1u << q;
            }
        }
    *out = r;
    return RPQ_OK;
}

}  // extern "C"

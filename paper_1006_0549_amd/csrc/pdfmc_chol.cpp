// Nested-dissection supernodal Cholesky factorization on the host.
//
// Ordering: recursive coordinate bisection of the unknowns; the unknowns of
// one half that touch the other half form the separator, which is eliminated
// after both halves. Factorization: multifrontal, in the order the dissection
// creates the supernodes (children first): each supernode's dense front holds
// its own columns of K plus its children's update matrices; the partial
// Cholesky factorization of the front gives L11 and L21 and the update matrix
// passed to the parent.
#include "pdfmc_chol.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace pdfmc {

namespace {

// K with the off-diagonal entries of row and column `pin` removed
CsrH decouple(const CsrH& K, int pin)
{
    CsrH M;
    M.n = M.m = K.n;
    M.ptr.assign(K.n + 1, 0);
    for (int i = 0; i < K.n; ++i) {
        for (int k = K.ptr[i]; k < K.ptr[i + 1]; ++k) {
            const int j = K.col[k];
            if ((i == pin || j == pin) && i != j) continue;
            M.col.push_back(j);
            M.val.push_back(K.val[k]);
        }
        M.ptr[i + 1] = (int)M.col.size();
    }
    return M;
}

struct Dissection {
    const CsrH& A;
    const std::vector<double>& x;
    const std::vector<double>& y;
    int leaf;
    std::vector<int> stamp;
    int cur = 0;
    std::vector<CholNode>& nodes;

    Dissection(const CsrH& A_, const std::vector<double>& x_, const std::vector<double>& y_, int leaf_,
               std::vector<CholNode>& nodes_)
        : A(A_), x(x_), y(y_), leaf(leaf_), stamp(A_.n, 0), nodes(nodes_) {}

    int add(std::vector<int> vars, std::vector<int> children)
    {
        CholNode s;
        s.vars = std::move(vars);
        s.children = std::move(children);
        nodes.push_back(std::move(s));
        return (int)nodes.size() - 1;
    }

    // unknowns of `side` with a neighbour carrying the current stamp
    std::vector<int> touching(const std::vector<int>& side) const
    {
        std::vector<int> out;
        for (int u : side)
            for (int k = A.ptr[u]; k < A.ptr[u + 1]; ++k)
                if (A.col[k] != u && stamp[A.col[k]] == cur) { out.push_back(u); break; }
        return out;
    }

    // Dissects `set`; returns the roots of the supernode forest built for it.
    std::vector<int> run(std::vector<int> set)
    {
        if (set.empty()) return {};
        if ((int)set.size() <= leaf) {
            std::sort(set.begin(), set.end());
            return {add(std::move(set), {})};
        }
        double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
        for (int u : set) {
            x0 = std::min(x0, x[u]); x1 = std::max(x1, x[u]);
            y0 = std::min(y0, y[u]); y1 = std::max(y1, y[u]);
        }
        const std::vector<double>& c = (x1 - x0 >= y1 - y0) ? x : y;
        const size_t mid = set.size() / 2;
        std::nth_element(set.begin(), set.begin() + mid, set.end(),
                         [&](int a, int b) { return c[a] < c[b] || (c[a] == c[b] && a < b); });
        std::vector<int> lo(set.begin(), set.begin() + mid), hi(set.begin() + mid, set.end());
        ++cur;
        for (int u : hi) stamp[u] = cur;
        std::vector<int> sep_lo = touching(lo);
        ++cur;
        for (int u : lo) stamp[u] = cur;
        std::vector<int> sep_hi = touching(hi);
        // the smaller boundary becomes the separator
        const bool take_lo = sep_lo.size() <= sep_hi.size();
        std::vector<int>& sep = take_lo ? sep_lo : sep_hi;
        std::vector<int>& side = take_lo ? lo : hi;
        ++cur;
        for (int u : sep) stamp[u] = cur;
        side.erase(std::remove_if(side.begin(), side.end(), [&](int u) { return stamp[u] == cur; }), side.end());
        std::vector<int> roots = run(std::move(lo));
        std::vector<int> r2 = run(std::move(hi));
        roots.insert(roots.end(), r2.begin(), r2.end());
        if (sep.empty()) return roots;
        std::sort(sep.begin(), sep.end());
        return {add(std::move(sep), std::move(roots))};
    }
};

}  // namespace

bool chol_factor(const CsrH& K, const std::vector<double>& x, const std::vector<double>& y, int pin, int leaf,
                 CholFactor& F, std::string& err)
{
    const int n = K.n;
    F = CholFactor();
    F.n = n;
    F.pin = pin;
    if (n <= 0) return true;
    const CsrH A = decouple(K, pin);
    {
        std::vector<int> all(n);
        std::iota(all.begin(), all.end(), 0);
        Dissection d(A, x, y, std::max(leaf, 4), F.nodes);
        d.run(std::move(all));
    }
    // elimination order: the supernodes in creation order (children first)
    std::vector<int> elim(n, -1), last(F.nodes.size());
    int pos = 0;
    for (size_t s = 0; s < F.nodes.size(); ++s) {
        for (int v : F.nodes[s].vars) elim[v] = pos++;
        last[s] = pos - 1;
    }
    if (pos != n) { err = "nested dissection lost unknowns"; return false; }
    std::vector<double> diag(n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
            if (A.col[k] == i) diag[i] = A.val[k];

    std::vector<int> fpos(n, -1);
    std::vector<std::vector<double>> upd(F.nodes.size());   // update matrices awaiting their parent
    for (size_t si = 0; si < F.nodes.size(); ++si) {
        CholNode& S = F.nodes[si];
        const int s = (int)S.vars.size();
        for (int i = 0; i < s; ++i) fpos[S.vars[i]] = i;
        // later variables reached: neighbours eliminated after this supernode
        // and what the children's update matrices reach
        std::vector<int>& str = S.str;
        auto reach = [&](int u) {
            if (fpos[u] < 0 && elim[u] > last[si]) { fpos[u] = s; str.push_back(u); }
        };
        for (int v : S.vars)
            for (int k = A.ptr[v]; k < A.ptr[v + 1]; ++k) reach(A.col[k]);
        for (int c : S.children)
            for (int u : F.nodes[c].str) {
                if (fpos[u] < 0 && elim[u] <= last[si]) {
                    err = "projection factor: inconsistent dissection";
                    return false;
                }
                reach(u);
            }
        std::sort(str.begin(), str.end(), [&](int a, int b) { return elim[a] < elim[b]; });
        const int m = (int)str.size(), f = s + m;
        for (int k = 0; k < m; ++k) fpos[str[k]] = s + k;
        // dense front, lower triangle, row-major
        std::vector<double> Fm((size_t)f * f, 0.0);
        for (int j = 0; j < s; ++j) {
            const int v = S.vars[j];
            for (int k = A.ptr[v]; k < A.ptr[v + 1]; ++k) {
                const int u = A.col[k];
                if (fpos[u] < 0 || elim[u] < elim[v]) continue;
                Fm[(size_t)fpos[u] * f + j] += A.val[k];
            }
        }
        for (int c : S.children) {
            const std::vector<int>& cs = F.nodes[c].str;
            const std::vector<double>& U = upd[c];
            const int mc = (int)cs.size();
            for (int a = 0; a < mc; ++a)
                for (int b = 0; b <= a; ++b) {
                    int i = fpos[cs[a]], j = fpos[cs[b]];
                    if (i < j) std::swap(i, j);
                    Fm[(size_t)i * f + j] += U[(size_t)a * mc + b];
                }
            std::vector<double>().swap(upd[c]);
        }
        // partial Cholesky factorization of the front: s pivots
        for (int k = 0; k < s; ++k) {
            double& p = Fm[(size_t)k * f + k];
            if (!(p > 1e-13 * std::fabs(diag[S.vars[k]]))) {
                err = "projection factor: pivot not positive (disconnected mesh?)";
                return false;
            }
            p = std::sqrt(p);
            for (int i = k + 1; i < f; ++i) Fm[(size_t)i * f + k] /= p;
            for (int j = k + 1; j < f; ++j) {
                const double ljk = Fm[(size_t)j * f + k];
                if (ljk == 0.0) continue;
                for (int i = j; i < f; ++i) Fm[(size_t)i * f + j] -= Fm[(size_t)i * f + k] * ljk;
            }
        }
        // L11^-1 by forward substitution, column by column
        S.linv.assign((size_t)s * s, 0.0);
        for (int j = 0; j < s; ++j) {
            S.linv[(size_t)j * s + j] = 1.0 / Fm[(size_t)j * f + j];
            for (int i = j + 1; i < s; ++i) {
                double t = 0.0;
                for (int k = j; k < i; ++k) t += Fm[(size_t)i * f + k] * S.linv[(size_t)k * s + j];
                S.linv[(size_t)i * s + j] = -t / Fm[(size_t)i * f + i];
            }
        }
        S.l21.assign((size_t)m * s, 0.0);
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < s; ++b) S.l21[(size_t)a * s + b] = Fm[(size_t)(s + a) * f + b];
        if (m > 0) {
            std::vector<double>& U = upd[si];
            U.assign((size_t)m * m, 0.0);
            for (int a = 0; a < m; ++a)
                for (int b = 0; b <= a; ++b) U[(size_t)a * m + b] = Fm[(size_t)(s + a) * f + (s + b)];
        }
        int h = 0;
        for (int c : S.children) h = std::max(h, F.nodes[c].height + 1);
        S.height = h;
        F.height = std::max(F.height, h);
        F.max_s = std::max(F.max_s, s);
        F.max_m = std::max(F.max_m, m);
        F.n_idx += s + m;
        F.n_val += (int64_t)s * s + (int64_t)m * s;
        for (int v : S.vars) fpos[v] = -1;
        for (int u : str) fpos[u] = -1;
    }
    return true;
}

}  // namespace pdfmc

// Smoothed-aggregation multigrid setup (host).
//
// Standard smoothed aggregation for a scalar elliptic operator whose
// near-null space is the constant vector:
//   strength   |a_ij| >= theta sqrt(|a_ii a_jj|)
//   aggregates three passes: root + strong neighbours; attach leftovers to
//              the aggregate they are most strongly tied to; group the rest
//   P_tent     one column per aggregate, entries 1/sqrt(|aggregate|)
//   P          (I - omega D_F^-1 A_F) P_tent, A_F = A with weak couplings
//              lumped onto the diagonal, omega = 4 / (3 rho(D_F^-1 A_F))
//   A_c        P^T A P, kept as a list of contributions so the coarse values
//              can be recomputed when A's values change.
// On the graded meshes the strength test keeps only the couplings across the
// thin near-wall cells, so the aggregates line up with them (semi-coarsening
// where the mesh is anisotropic).
#include "pdfmc_amg.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <tuple>

namespace pdfmc {

namespace {

std::vector<char> strength(const CsrH& A, const std::vector<int>& iso, double theta, std::vector<double>& diag)
{
    diag.assign(A.n, 0.0);
    for (int i = 0; i < A.n; ++i)
        for (int j = A.ptr[i]; j < A.ptr[i + 1]; ++j)
            if (A.col[j] == i) diag[i] = A.val[j];
    std::vector<char> S(A.col.size(), 0);
    for (int i = 0; i < A.n; ++i) {
        if (!iso.empty() && iso[i]) continue;
        for (int j = A.ptr[i]; j < A.ptr[i + 1]; ++j) {
            int c = A.col[j];
            if (c == i || (!iso.empty() && iso[c])) continue;
            if (std::fabs(A.val[j]) >= theta * std::sqrt(std::fabs(diag[i] * diag[c]))) S[j] = 1;
        }
    }
    return S;
}

int aggregate(const CsrH& A, const std::vector<char>& S, std::vector<int>& agg)
{
    const int n = A.n;
    agg.assign(n, -1);
    int na = 0;
    auto nstrong = [&](int i) {
        int k = 0;
        for (int j = A.ptr[i]; j < A.ptr[i + 1]; ++j) k += S[j];
        return k;
    };
    // pass 1: roots whose strong neighbourhood is entirely free
    for (int i = 0; i < n; ++i) {
        if (agg[i] >= 0 || nstrong(i) == 0) continue;
        bool free = true;
        for (int j = A.ptr[i]; j < A.ptr[i + 1] && free; ++j)
            if (S[j] && agg[A.col[j]] >= 0) free = false;
        if (!free) continue;
        agg[i] = na;
        for (int j = A.ptr[i]; j < A.ptr[i + 1]; ++j)
            if (S[j]) agg[A.col[j]] = na;
        ++na;
    }
    // pass 2: attach to the most strongly connected neighbouring aggregate
    std::vector<int> snap = agg;
    for (int i = 0; i < n; ++i) {
        if (snap[i] >= 0) continue;
        double best = 0.0;
        int ba = -1;
        for (int j = A.ptr[i]; j < A.ptr[i + 1]; ++j)
            if (S[j] && snap[A.col[j]] >= 0 && std::fabs(A.val[j]) > best) { best = std::fabs(A.val[j]); ba = snap[A.col[j]]; }
        if (ba >= 0) agg[i] = ba;
    }
    // pass 3: remaining nodes with strong couplings form new aggregates
    for (int i = 0; i < n; ++i) {
        if (agg[i] >= 0 || nstrong(i) == 0) continue;
        agg[i] = na;
        for (int j = A.ptr[i]; j < A.ptr[i + 1]; ++j)
            if (S[j] && agg[A.col[j]] < 0) agg[A.col[j]] = na;
        ++na;
    }
    return na;
}

void transpose(const CsrH& P, CsrH& R)
{
    R.n = P.m; R.m = P.n;
    R.ptr.assign(R.n + 1, 0);
    for (int c : P.col) R.ptr[c + 1]++;
    for (int i = 0; i < R.n; ++i) R.ptr[i + 1] += R.ptr[i];
    R.col.assign(P.col.size(), 0);
    R.val.assign(P.col.size(), 0.0);
    std::vector<int> fill(R.ptr.begin(), R.ptr.end() - 1);
    for (int i = 0; i < P.n; ++i)
        for (int j = P.ptr[i]; j < P.ptr[i + 1]; ++j) {
            int q = fill[P.col[j]]++;
            R.col[q] = i;
            R.val[q] = P.val[j];
        }
}

}  // namespace

void amg_setup(const CsrH& A0, const std::vector<int>& isolated, AmgH& H, int max_coarse, int max_levels)
{
    H.lv.clear();
    H.lv.emplace_back();
    H.lv[0].A = A0;
    std::vector<int> iso = isolated;
    const double theta = 0.1;
    while ((int)H.lv.size() < max_levels && H.lv.back().A.n > max_coarse) {
        AmgLevelH& L = H.lv.back();
        const CsrH& A = L.A;
        std::vector<double> diag;
        std::vector<char> S = strength(A, iso, theta, diag);
        std::vector<int> agg;
        int na = aggregate(A, S, agg);
        if (na == 0 || na >= A.n) break;
        std::vector<int> size(na, 0);
        for (int a : agg) if (a >= 0) size[a]++;
        // filtered operator: weak couplings lumped onto the diagonal
        std::vector<double> dF(A.n, 0.0);
        for (int i = 0; i < A.n; ++i) {
            double d = 0.0;
            for (int j = A.ptr[i]; j < A.ptr[i + 1]; ++j) {
                int c = A.col[j];
                if (c == i) d += A.val[j];
                else if (!S[j]) d += A.val[j];
            }
            dF[i] = d;
        }
        auto applyDinvAF = [&](const std::vector<double>& x, std::vector<double>& y) {
            for (int i = 0; i < A.n; ++i) {
                double s = dF[i] * x[i];
                for (int j = A.ptr[i]; j < A.ptr[i + 1]; ++j)
                    if (S[j]) s += A.val[j] * x[A.col[j]];
                y[i] = (std::fabs(dF[i]) > 0.0) ? s / dF[i] : 0.0;
            }
        };
        // spectral radius of D_F^-1 A_F by power iteration
        std::vector<double> v(A.n), w(A.n);
        for (int i = 0; i < A.n; ++i) v[i] = 1.0 + 0.37 * std::sin(1.3 * i);
        double rho = 1.0;
        for (int it = 0; it < 25; ++it) {
            applyDinvAF(v, w);
            double nw = 0.0, nv = 0.0;
            for (int i = 0; i < A.n; ++i) { nw += w[i] * w[i]; nv += v[i] * v[i]; }
            rho = std::sqrt(nw / std::max(nv, 1e-300));
            double s = 1.0 / std::sqrt(std::max(nw, 1e-300));
            for (int i = 0; i < A.n; ++i) v[i] = w[i] * s;
        }
        const double omega = 4.0 / (3.0 * std::max(rho, 1e-12));
        // P = P_tent - omega D_F^-1 A_F P_tent, row by row
        CsrH& P = L.P;
        P.n = A.n; P.m = na;
        P.ptr.assign(A.n + 1, 0);
        P.col.clear(); P.val.clear();
        std::vector<double> acc(na, 0.0);
        std::vector<int> touched;
        for (int i = 0; i < A.n; ++i) {
            touched.clear();
            auto add = [&](int c, double x) {
                if (acc[c] == 0.0) touched.push_back(c);
                acc[c] += x;
                if (acc[c] == 0.0) acc[c] = 1e-300;   // keep it in the pattern
            };
            if (agg[i] >= 0) add(agg[i], 1.0 / std::sqrt((double)size[agg[i]]));
            if (std::fabs(dF[i]) > 0.0) {
                double f = -omega / dF[i];
                if (agg[i] >= 0) add(agg[i], f * dF[i] / std::sqrt((double)size[agg[i]]));
                for (int j = A.ptr[i]; j < A.ptr[i + 1]; ++j) {
                    int c = A.col[j];
                    if (!S[j] || agg[c] < 0) continue;
                    add(agg[c], f * A.val[j] / std::sqrt((double)size[agg[c]]));
                }
            }
            std::sort(touched.begin(), touched.end());
            for (int c : touched) {
                P.col.push_back(c);
                P.val.push_back(acc[c]);
                acc[c] = 0.0;
            }
            P.ptr[i + 1] = (int)P.col.size();
        }
        transpose(P, L.R);
        // Galerkin product with its contribution lists
        std::vector<std::tuple<int, int, int, double>> contrib;   // (I, J, fine nz, coef)
        for (int i = 0; i < A.n; ++i)
            for (int q = A.ptr[i]; q < A.ptr[i + 1]; ++q) {
                int j = A.col[q];
                for (int a = P.ptr[i]; a < P.ptr[i + 1]; ++a)
                    for (int b = P.ptr[j]; b < P.ptr[j + 1]; ++b)
                        contrib.emplace_back(P.col[a], P.col[b], q, P.val[a] * P.val[b]);
            }
        std::sort(contrib.begin(), contrib.end(), [](const auto& x, const auto& y) {
            if (std::get<0>(x) != std::get<0>(y)) return std::get<0>(x) < std::get<0>(y);
            if (std::get<1>(x) != std::get<1>(y)) return std::get<1>(x) < std::get<1>(y);
            return std::get<2>(x) < std::get<2>(y);
        });
        AmgLevelH next;
        CsrH& C = next.A;
        C.n = na; C.m = na;
        C.ptr.assign(na + 1, 0);
        L.gptr.assign(1, 0);
        L.gidx.clear(); L.gcoef.clear();
        for (size_t k = 0; k < contrib.size();) {
            size_t e = k;
            int I = std::get<0>(contrib[k]), J = std::get<1>(contrib[k]);
            double s = 0.0;
            while (e < contrib.size() && std::get<0>(contrib[e]) == I && std::get<1>(contrib[e]) == J) {
                L.gidx.push_back(std::get<2>(contrib[e]));
                L.gcoef.push_back(std::get<3>(contrib[e]));
                s += std::get<3>(contrib[e]) * A.val[std::get<2>(contrib[e])];
                ++e;
            }
            C.col.push_back(J);
            C.val.push_back(s);
            C.ptr[I + 1]++;
            L.gptr.push_back((int)L.gidx.size());
            k = e;
        }
        for (int i = 0; i < na; ++i) C.ptr[i + 1] += C.ptr[i];
        // every coarse row holds its diagonal (aggregates are non-empty)
        iso.assign(na, 0);
        H.lv.push_back(std::move(next));
    }
}

void to_ell(const CsrH& A, bool pad_self, EllH& E)
{
    E.n = A.n;
    E.w = 0;
    for (int i = 0; i < A.n; ++i) E.w = std::max(E.w, A.ptr[i + 1] - A.ptr[i]);
    E.w = std::max(E.w, 1);
    E.w = (E.w + 3) / 4 * 4;   // the device loops take four entries at a time
    E.col.assign((size_t)E.w * A.n, 0);
    E.val.assign((size_t)E.w * A.n, 0.0);
    E.len.assign(A.n, 0);
    E.map.assign(A.col.size(), 0);
    for (int i = 0; i < A.n; ++i) {
        E.len[i] = A.ptr[i + 1] - A.ptr[i];
        for (int k = 0; k < E.w; ++k) {
            const size_t at = (size_t)k * A.n + i;
            const int j = A.ptr[i] + k;
            if (j < A.ptr[i + 1]) {
                E.col[at] = A.col[j];
                E.val[at] = A.val[j];
                E.map[j] = (int)at;
            } else {
                E.col[at] = pad_self ? i : 0;
            }
        }
    }
}

}  // namespace pdfmc

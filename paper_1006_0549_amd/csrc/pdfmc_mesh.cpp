// Host-side derivation of the grid tables of one case (Sec. I: the grid is
// used for statistics, Eulerian solves and tracking).
//   - element records of the barycentric formula (R-05),
//   - neighbours across edge k (opposite vertex k, R-04),
//   - periodic partners, matched by exactly equal coordinates after the
//     boundary's shift (R-15), and merged periodic images (R-33),
//   - lumped node areas, node -> element incidence, wall normals (R-19),
//   - the sparsity pattern of the P1 Galerkin matrices.
#include "pdfmc_mesh.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <tuple>

namespace pdfmc {

static std::string fmt(const char* f, long a, long b = 0)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, f, a, b);
    return buf;
}

int derive_mesh(const pdfmc_mesh_desc& d, MeshHost& m, std::string& err)
{
    if (d.n_nodes < 3 || d.n_elems < 1 || !d.xy || !d.tri || !d.edge_tag || d.n_bc < 0 || (d.n_bc > 0 && !d.bc)) {
        err = "mesh: missing arrays or empty mesh";
        return PDFMC_E_INVALID;
    }
    if (d.n_elems >= (1 << 23)) {
        // the scatter sorts a wavefront's particles on (element << 9 | bin << 6 | lane) in 32 bits
        err = "mesh: a case holds at most 2^23 - 1 elements";
        return PDFMC_E_INVALID;
    }
    const int nn = d.n_nodes, ne = d.n_elems;
    m.nn = nn; m.ne = ne;
    m.x.resize(nn); m.y.resize(nn);
    for (int i = 0; i < nn; ++i) { m.x[i] = d.xy[2 * i]; m.y[i] = d.xy[2 * i + 1]; }
    m.tri.assign(d.tri, d.tri + 3 * (size_t)ne);
    m.tag.assign(d.edge_tag, d.edge_tag + 3 * (size_t)ne);
    m.bc.assign(d.bc, d.bc + d.n_bc);
    for (int i = 0; i < 3 * ne; ++i) {
        if (m.tri[i] < 0 || m.tri[i] >= nn) { err = fmt("mesh: element %ld references node %ld", i / 3, m.tri[i]); return PDFMC_E_MESH; }
        if (m.tag[i] < -1 || m.tag[i] >= d.n_bc) { err = fmt("mesh: element %ld has edge tag %ld", i / 3, m.tag[i]); return PDFMC_E_MESH; }
    }
    for (const auto& b : m.bc)
        if (b.type != PDFMC_BC_WALL && b.type != PDFMC_BC_PERIODIC) { err = "mesh: unknown boundary type"; return PDFMC_E_MESH; }

    // records (R-05): D as two products and one subtraction
    m.rec.resize(8 * (size_t)ne);
    m.area.resize(ne);
    for (int e = 0; e < ne; ++e) {
        const int* v = &m.tri[3 * e];
        double X[3] = {m.x[v[0]], m.x[v[1]], m.x[v[2]]}, Y[3] = {m.y[v[0]], m.y[v[1]], m.y[v[2]]};
        double p = (X[1] - X[0]) * (Y[2] - Y[0]);
        double q = (X[2] - X[0]) * (Y[1] - Y[0]);
        double D = p - q;
        if (!(D > 0.0)) { err = fmt("mesh: element %ld is not counter-clockwise", e); return PDFMC_E_MESH; }
        double* r = &m.rec[8 * (size_t)e];
        r[0] = X[0]; r[1] = Y[0];
        for (int k = 0; k < 3; ++k) {
            int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
            r[2 + k] = (Y[k1] - Y[k2]) / D;
            r[5 + k] = (X[k2] - X[k1]) / D;
        }
        m.area[e] = 0.5 * D;
    }

    // neighbours
    std::vector<std::tuple<int64_t, int, int>> edges;   // (key, e, k)
    edges.reserve(3 * (size_t)ne);
    for (int e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) {
            int a = m.tri[3 * e + (k + 1) % 3], b = m.tri[3 * e + (k + 2) % 3];
            int64_t key = (int64_t)std::min(a, b) * nn + std::max(a, b);
            edges.emplace_back(key, e, k);
        }
    std::sort(edges.begin(), edges.end());
    m.nbr.assign(3 * (size_t)ne, -1);
    m.partner.assign(3 * (size_t)ne, -1);
    for (size_t i = 0; i < edges.size();) {
        size_t j = i;
        while (j < edges.size() && std::get<0>(edges[j]) == std::get<0>(edges[i])) ++j;
        if (j - i == 1) {
            auto [key, e, k] = edges[i];
            if (m.tag[3 * e + k] < 0) { err = fmt("mesh: boundary edge of element %ld has no tag", e); return PDFMC_E_MESH; }
        } else if (j - i == 2) {
            auto [k0, e1, l1] = edges[i];
            auto [k1, e2, l2] = edges[i + 1];
            int a1 = m.tri[3 * e1 + (l1 + 1) % 3], b1 = m.tri[3 * e1 + (l1 + 2) % 3];
            int a2 = m.tri[3 * e2 + (l2 + 1) % 3], b2 = m.tri[3 * e2 + (l2 + 2) % 3];
            if (a1 != b2 || b1 != a2) { err = fmt("mesh: inconsistent orientation at elements %ld, %ld", e1, e2); return PDFMC_E_MESH; }
            if (m.tag[3 * e1 + l1] >= 0 || m.tag[3 * e2 + l2] >= 0) { err = fmt("mesh: interior edge of element %ld carries a boundary tag", e1); return PDFMC_E_MESH; }
            m.nbr[3 * e1 + l1] = e2;
            m.nbr[3 * e2 + l2] = e1;
        } else {
            err = fmt("mesh: non-manifold edge shared by %ld elements", (long)(j - i));
            return PDFMC_E_MESH;
        }
        i = j;
    }

    // periodic partners by exact coordinates
    std::map<std::pair<double, double>, std::vector<std::pair<int, int>>> by_start;   // start vertex -> (e,k)
    for (int e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) {
            int t = m.tag[3 * e + k];
            if (t < 0 || m.bc[t].type != PDFMC_BC_PERIODIC) continue;
            int a = m.tri[3 * e + (k + 1) % 3];
            by_start[{m.x[a], m.y[a]}].push_back({e, k});
        }
    std::vector<int> par(nn);
    std::iota(par.begin(), par.end(), 0);
    auto find = [&](int i) { while (par[i] != i) i = par[i]; return i; };
    auto unite = [&](int i, int j) {
        int a = find(i), b = find(j);
        if (a == b) return;
        if (a < b) par[b] = a; else par[a] = b;
    };
    for (int e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) {
            int t = m.tag[3 * e + k];
            if (t < 0 || m.bc[t].type != PDFMC_BC_PERIODIC) continue;
            int a = m.tri[3 * e + (k + 1) % 3], b = m.tri[3 * e + (k + 2) % 3];
            double sx = m.bc[t].shift[0], sy = m.bc[t].shift[1];
            // partner edge runs from (b + s) to (a + s)
            auto it = by_start.find({m.x[b] + sx, m.y[b] + sy});
            int pe = -1, pk = -1;
            if (it != by_start.end())
                for (auto [e2, k2] : it->second) {
                    int b2 = m.tri[3 * e2 + (k2 + 2) % 3];
                    if (m.x[b2] == m.x[a] + sx && m.y[b2] == m.y[a] + sy) { pe = e2; pk = k2; break; }
                }
            if (pe < 0) { err = fmt("mesh: periodic edge of element %ld has no partner", e); return PDFMC_E_MESH; }
            int t2 = m.tag[3 * pe + pk];
            if (m.bc[t2].shift[0] != -sx || m.bc[t2].shift[1] != -sy) {
                err = fmt("mesh: periodic boundaries %ld and %ld have shifts that are not opposite", t, t2);
                return PDFMC_E_MESH;
            }
            m.partner[3 * e + k] = pe;
            unite(a, m.tri[3 * pe + (pk + 2) % 3]);
            unite(b, m.tri[3 * pe + (pk + 1) % 3]);
        }

    // statistics nodes
    m.snode.assign(nn, -1);
    m.rep.clear();
    for (int i = 0; i < nn; ++i)
        if (find(i) == i) { m.snode[i] = (int)m.rep.size(); m.rep.push_back(i); }
    for (int i = 0; i < nn; ++i) m.snode[i] = m.snode[find(i)];
    m.nsn = (int)m.rep.size();
    m.tri_s.resize(3 * (size_t)ne);
    m.vol.assign(m.nsn, 0.0);
    for (int e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) {
            int s = m.snode[m.tri[3 * e + k]];
            m.tri_s[3 * e + k] = s;
            m.vol[s] += m.area[e] / 3.0;
        }
    // incidence, increasing (element, vertex)
    m.inc_ptr.assign(m.nsn + 1, 0);
    for (int i = 0; i < 3 * ne; ++i) m.inc_ptr[m.tri_s[i] + 1]++;
    for (int s = 0; s < m.nsn; ++s) m.inc_ptr[s + 1] += m.inc_ptr[s];
    m.inc.assign(3 * (size_t)ne, 0);
    {
        std::vector<int> fill(m.inc_ptr.begin(), m.inc_ptr.end() - 1);
        for (int i = 0; i < 3 * ne; ++i) m.inc[fill[m.tri_s[i]]++] = i;
    }
    // wall normals
    m.is_wall.assign(m.nsn, 0);
    m.wnx.assign(m.nsn, 0.0);
    m.wny.assign(m.nsn, 0.0);
    for (int e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) {
            int t = m.tag[3 * e + k];
            if (t < 0 || m.bc[t].type != PDFMC_BC_WALL) continue;
            int a = m.tri[3 * e + (k + 1) % 3], b = m.tri[3 * e + (k + 2) % 3];
            double dx = m.x[b] - m.x[a], dy = m.y[b] - m.y[a];
            double L = std::sqrt(dx * dx + dy * dy);
            for (int s : {m.snode[a], m.snode[b]}) {
                m.is_wall[s] = 1;
                m.wnx[s] += dy / L;
                m.wny[s] += -dx / L;
            }
        }
    for (int s = 0; s < m.nsn; ++s)
        if (m.is_wall[s]) {
            double L = std::sqrt(m.wnx[s] * m.wnx[s] + m.wny[s] * m.wny[s]);
            m.wnx[s] /= L; m.wny[s] /= L;
        }
    // Galerkin sparsity pattern and the positions of each (row, vertex) pair
    m.csr_ptr.assign(m.nsn + 1, 0);
    m.csr_col.clear();
    std::vector<int> cols;
    for (int s = 0; s < m.nsn; ++s) {
        cols.clear();
        for (int j = m.inc_ptr[s]; j < m.inc_ptr[s + 1]; ++j) {
            int e = m.inc[j] / 3;
            for (int k = 0; k < 3; ++k) cols.push_back(m.tri_s[3 * e + k]);
        }
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        m.csr_col.insert(m.csr_col.end(), cols.begin(), cols.end());
        m.csr_ptr[s + 1] = (int)m.csr_col.size();
    }
    m.incpos.assign(3 * m.inc.size(), 0);
    for (int s = 0; s < m.nsn; ++s)
        for (int j = m.inc_ptr[s]; j < m.inc_ptr[s + 1]; ++j) {
            int e = m.inc[j] / 3;
            for (int k = 0; k < 3; ++k) {
                int col = m.tri_s[3 * e + k];
                auto first = m.csr_col.begin() + m.csr_ptr[s], last = m.csr_col.begin() + m.csr_ptr[s + 1];
                m.incpos[3 * (size_t)j + k] = (int)(std::lower_bound(first, last, col) - m.csr_col.begin());
            }
        }
    return PDFMC_OK;
}

}  // namespace pdfmc

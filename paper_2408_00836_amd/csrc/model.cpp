// model.cpp -- lattice, bonds, hopping groups and start state of the
// Hubbard model of Eq. (1), generalised per bond and site as in Eq. (2),
// (15) and (16).  Host only; no GPU calls.
#include <cmath>
#include <map>
#include <set>
#include <string>

#include "hubvqe.hpp"

namespace hv {

namespace {

enum { H1 = 0, V1 = 1, H2 = 2, V2 = 3 };

struct RawBond {
    int i, j, cls;
};

// Canonical bond order and the default commuting split of Eq. (7): horizontal
// bonds by start-column parity (h1 even, h2 odd), vertical bonds by start-row
// parity (v1, v2); a direction of length 2 with transverse length >= 3 splits
// by the transverse parity so that each group stays a matching.
std::vector<RawBond> lattice_bonds(int nx, int ny, bool px, bool py)
{
    std::vector<RawBond> out;
    const bool h_by_row = (ny == 2 && nx >= 3);
    const bool v_by_col = (nx == 2 && ny >= 3);
    for (int x = 0; x < nx; ++x) {
        for (int y = 0; y < ny; ++y) {
            int yn;
            if (y + 1 < ny)
                yn = y + 1;
            else if (py)
                yn = 0;
            else
                continue;
            int par = (h_by_row ? x : y) & 1;
            out.push_back({x * ny + y, x * ny + yn, par ? H2 : H1});
        }
    }
    for (int x = 0; x < nx; ++x) {
        for (int y = 0; y < ny; ++y) {
            int xn;
            if (x + 1 < nx)
                xn = x + 1;
            else if (px)
                xn = 0;
            else
                continue;
            int par = (v_by_col ? y : x) & 1;
            out.push_back({x * ny + y, xn * ny + y, par ? V2 : V1});
        }
    }
    return out;
}

}  // namespace

namespace {

// Groups, per-bond and per-site constants, validation and start state shared
// by the lattice and the graph forms.  spin[s]: start spin of site s.
std::string finish_model(const std::vector<RawBond> &raw, const double *t, double U,
                         const double *V, const double *eps, const int32_t *groups,
                         const std::vector<int> &spin, Model &m)
{
    if (!std::isfinite(U))
        return "U must be finite";
    m.nq = 2 * m.ns;
    m.U = U;
    m.nb = (int)raw.size();
    if (m.nb > kMaxBonds)
        return "too many bonds";
    std::vector<int> cls(m.nb);
    for (int b = 0; b < m.nb; ++b) {
        cls[b] = raw[b].cls;
        if (groups) {
            if (groups[b] < 0)
                return "bond_group ids must be >= 0";
            cls[b] = groups[b];
        }
    }
    // Every group must be a matching: its terms then act on disjoint modes and
    // commute, so the group exponential is the product of the term ones.
    std::map<int, std::set<int>> used;
    for (int b = 0; b < m.nb; ++b) {
        std::set<int> &u = used[cls[b]];
        if (u.count(raw[b].i) || u.count(raw[b].j))
            return "hopping group " + std::to_string(cls[b]) +
                   " is not a matching (a site appears in two of its bonds)";
        u.insert(raw[b].i);
        u.insert(raw[b].j);
    }
    std::map<int, int> slot_of;   // group id -> slot 1..G in increasing id
    for (auto &kv : used)
        slot_of[kv.first] = 0;
    int s = 0;
    for (auto &kv : slot_of)
        kv.second = ++s;
    m.ngroups = s;

    m.bi.resize(m.nb);
    m.bj.resize(m.nb);
    m.slot.resize(m.nb);
    m.t.assign(m.nb, 1.0);
    m.V.assign(m.nb, 0.0);
    m.eps.assign(m.ns, 0.0);
    for (int b = 0; b < m.nb; ++b) {
        m.bi[b] = raw[b].i;
        m.bj[b] = raw[b].j;
        m.slot[b] = slot_of[cls[b]];
        if (t)
            m.t[b] = t[b];
        if (V)
            m.V[b] = V[b];
        if (!std::isfinite(m.t[b]) || !std::isfinite(m.V[b]))
            return "t_bond and V_bond must be finite";
        if (m.V[b] != 0.0)
            m.general = true;
    }
    for (int i = 0; i < m.ns; ++i) {
        if (eps)
            m.eps[i] = eps[i];
        if (!std::isfinite(m.eps[i]))
            return "eps_site must be finite";
        if (m.eps[i] != 0.0)
            m.general = true;
    }
    m.neel = 0;
    for (int site = 0; site < m.ns; ++site)
        m.neel |= (uint64_t)1 << m.qubit(site, spin[site]);
    return "";
}

}  // namespace

std::string build_model(int nx, int ny, int px, int py, const double *t, double U,
                        const double *V, const double *eps, const int32_t *groups, Model &m)
{
    if (nx < 1 || ny < 1)
        return "nx and ny must be >= 1";
    if ((long)nx * ny > kMaxSites)
        return "at most 16 sites (32 qubits)";
    if (px && nx < 3)
        return "periodic_x needs nx >= 3";
    if (py && ny < 3)
        return "periodic_y needs ny >= 3";
    m = Model();
    m.nx = nx;
    m.ny = ny;
    m.px = px ? 1 : 0;
    m.py = py ? 1 : 0;
    m.ns = nx * ny;
    // Checkerboard start (Sec. 2.1): spin up where x+y is even, down otherwise.
    std::vector<int> spin(m.ns);
    for (int x = 0; x < nx; ++x)
        for (int y = 0; y < ny; ++y)
            spin[x * ny + y] = ((x + y) & 1) ? 1 : 0;
    return finish_model(lattice_bonds(nx, ny, px != 0, py != 0), t, U, V, eps, groups, spin, m);
}

std::string build_graph_model(int n_sites, int n_bonds, const int32_t *bi, const int32_t *bj,
                              const double *t, double U, const double *V, const double *eps,
                              const int32_t *groups, const int32_t *site_spin, Model &m)
{
    if (n_sites < 1 || n_sites > kMaxSites)
        return "n_sites must be in [1, 16] (at most 32 qubits)";
    if (n_bonds < 0 || n_bonds > kMaxBonds)
        return "n_bonds must be in [0, 64]";
    if (n_bonds > 0 && (!bi || !bj))
        return "bond_i and bond_j are required when n_bonds > 0";
    std::vector<RawBond> raw;
    std::set<std::pair<int, int>> seen;
    // default groups: in bond order, the lowest group whose bonds use neither site
    std::vector<std::set<int>> used;
    for (int b = 0; b < n_bonds; ++b) {
        const int i = bi[b], j = bj[b];
        if (i < 0 || i >= n_sites || j < 0 || j >= n_sites || i == j)
            return "bond " + std::to_string(b) + " has a bad site";
        if (!seen.insert({std::min(i, j), std::max(i, j)}).second)
            return "bond " + std::to_string(b) + " is listed twice";
        size_t g = 0;
        while (g < used.size() && (used[g].count(i) || used[g].count(j)))
            ++g;
        if (g == used.size())
            used.emplace_back();
        used[g].insert(i);
        used[g].insert(j);
        raw.push_back({i, j, (int)g});
    }
    std::vector<int> spin(n_sites);
    for (int s = 0; s < n_sites; ++s) {
        spin[s] = site_spin ? site_spin[s] : (s & 1);
        if (spin[s] != 0 && spin[s] != 1)
            return "site_spin entries must be 0 (up) or 1 (down)";
    }
    m = Model();
    m.nx = 1;
    m.ny = n_sites;
    m.ns = n_sites;
    return finish_model(raw, t, U, V, eps, groups, spin, m);
}

}  // namespace hv

// Host-side symbolic set-up, once per mesh: node graph and 4x4-block BSR
// pattern, element colouring and element-to-block maps (for colour-by-colour
// atomic-free assembly), outlet slots, the distance-2 pattern of
// S_hat = D - C diag(A)^{-1} B (Sec. 3.1), and the AMG aggregates with their
// Galerkin gather lists.  Integer work only; no device calls.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <set>

#include "internal.h"

namespace ns {
namespace {

int64_t find_in_row(const Csr& c, int32_t i, int32_t j) {
    auto b = c.col.begin() + c.rp[i], e = c.col.begin() + c.rp[i + 1];
    auto it = std::lower_bound(b, e, j);
    if (it == e || *it != j) return -1;
    return it - c.col.begin();
}

// Greedy pairwise matching in ascending node order: an unmatched node takes
// its first (lowest index) unmatched neighbour, or stays single; coarse ids in
// creation order.  Self entries of the pattern are skipped.
std::vector<int32_t> greedy_matching(const Csr& c, int& nc) {
    std::vector<int32_t> agg(c.n, -1);
    nc = 0;
    for (int i = 0; i < c.n; ++i) {
        if (agg[i] != -1) continue;
        agg[i] = nc;
        for (int k = c.rp[i]; k < c.rp[i + 1]; ++k) {
            int j = c.col[k];
            if (j != i && agg[j] == -1) {
                agg[j] = nc;
                break;
            }
        }
        ++nc;
    }
    return agg;
}

// Members of every group: CSR (ptr [ng+1], items ascending within a group).
static void group_lists(const std::vector<int32_t>& grp, int ng, std::vector<int32_t>& ptr,
                        std::vector<int32_t>& items) {
    ptr.assign(ng + 1, 0);
    for (int32_t g : grp) ptr[g + 1]++;
    for (int c = 0; c < ng; ++c) ptr[c + 1] += ptr[c];
    items.resize(grp.size());
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (size_t i = 0; i < grp.size(); ++i) items[fill[grp[i]]++] = (int32_t)i;
}

// Quotient pattern: (I,J) present when some fine (i,j) maps to it (rows built
// one coarse node at a time from its members, columns sorted).
Csr quotient(const Csr& c, const std::vector<int32_t>& agg, int nc) {
    std::vector<int32_t> ptr, mem;
    group_lists(agg, nc, ptr, mem);
    Csr q;
    q.n = nc;
    q.rp.assign(nc + 1, 0);
    q.col.reserve(c.col.size() / 2);
    std::vector<int32_t> mark(nc, -1), row;
    for (int I = 0; I < nc; ++I) {
        row.clear();
        for (int t = ptr[I]; t < ptr[I + 1]; ++t) {
            const int i = mem[t];
            for (int k = c.rp[i]; k < c.rp[i + 1]; ++k) {
                const int J = agg[c.col[k]];
                if (mark[J] != I) {
                    mark[J] = I;
                    row.push_back(J);
                }
            }
        }
        std::sort(row.begin(), row.end());
        q.col.insert(q.col.end(), row.begin(), row.end());
        q.rp[I + 1] = (int32_t)q.col.size();
    }
    q.col.shrink_to_fit();
    return q;
}

// Gather list: every fine nnz k is appended (ascending k) to the list of the
// coarse nnz it sums into.  The target of k is looked up through the
// positions of coarse row agg[i]'s columns, set once per coarse row.
void gather_lists(const Csr& fine, const Csr& coarse, const std::vector<int32_t>& agg,
                  std::vector<int32_t>& gptr, std::vector<int32_t>& gidx) {
    std::vector<int32_t> ptr, mem;
    group_lists(agg, coarse.n, ptr, mem);
    std::vector<int32_t> tgt(fine.col.size());
    std::vector<int32_t> pos(coarse.n, -1);
    gptr.assign(coarse.col.size() + 1, 0);
    for (int I = 0; I < coarse.n; ++I) {
        for (int q = coarse.rp[I]; q < coarse.rp[I + 1]; ++q) pos[coarse.col[q]] = q;
        for (int t = ptr[I]; t < ptr[I + 1]; ++t) {
            const int i = mem[t];
            for (int k = fine.rp[i]; k < fine.rp[i + 1]; ++k) {
                const int32_t q = pos[agg[fine.col[k]]];
                tgt[k] = q;
                gptr[q + 1]++;
            }
        }
    }
    for (size_t q = 0; q < coarse.col.size(); ++q) gptr[q + 1] += gptr[q];
    gidx.resize(fine.col.size());
    std::vector<int32_t> fill(gptr.begin(), gptr.end() - 1);
    for (size_t k = 0; k < fine.col.size(); ++k) gidx[fill[tgt[k]]++] = (int32_t)k;
}

// Greedy first-fit colouring of items that touch `per` nodes each.
int greedy_colors(int n_items, int per, const int32_t* nodes, int n_nodes, std::vector<int32_t>& color) {
    const int W = 4;  // 256 colours max
    std::vector<uint64_t> used((size_t)n_nodes * W, 0);
    color.assign(n_items, -1);
    int ncol = 0;
    for (int e = 0; e < n_items; ++e) {
        uint64_t m[W] = {0, 0, 0, 0};
        for (int a = 0; a < per; ++a)
            for (int w = 0; w < W; ++w) m[w] |= used[(size_t)nodes[e * per + a] * W + w];
        int c = -1;
        for (int w = 0; w < W && c < 0; ++w)
            if (~m[w]) c = w * 64 + __builtin_ctzll(~m[w]);
        if (c < 0) return -1;
        color[e] = c;
        ncol = std::max(ncol, c + 1);
        for (int a = 0; a < per; ++a) used[(size_t)nodes[e * per + a] * W + c / 64] |= (1ull << (c % 64));
    }
    return ncol;
}

}  // namespace

std::string build_symbolic(const ns_mesh* m, const ns_ctx_opts& o, Symbolic& S) {
    const int N = m->n_nodes, E = m->n_elems, NO = m->n_outlets;
    if (N <= 0 || E <= 0 || NO < 0) return "mesh sizes must be positive";
    if (!m->h_xyz || !m->h_tets || !m->h_dirichlet) return "mesh arrays missing";
    if (NO > 0 && (!m->h_outlet_ptr || !m->h_faces)) return "outlet arrays missing";
    S.N = N;
    S.E = E;
    S.n_out = NO;
    for (int64_t k = 0; k < (int64_t)E * 4; ++k)
        if (m->h_tets[k] < 0 || m->h_tets[k] >= N) return "tetrahedron vertex index out of range";

    // node -> element incidence (elements ascending per node)
    std::vector<int32_t> nptr, nelem;
    {
        std::vector<int32_t> vert(m->h_tets, m->h_tets + (size_t)E * 4);
        group_lists(vert, N, nptr, nelem);  // items: element slots 4e+a
    }
    // node graph (P1: nodes sharing an element), with the diagonal
    {
        Csr& g = S.g;
        g.n = N;
        g.rp.assign(N + 1, 0);
        g.col.reserve((size_t)N * 16);
        std::vector<int32_t> mark(N, -1), row;
        for (int i = 0; i < N; ++i) {
            row.clear();
            for (int t = nptr[i]; t < nptr[i + 1]; ++t) {
                const int32_t* tet = m->h_tets + 4 * (size_t)(nelem[t] / 4);
                for (int b = 0; b < 4; ++b)
                    if (mark[tet[b]] != i) {
                        mark[tet[b]] = i;
                        row.push_back(tet[b]);
                    }
            }
            std::sort(row.begin(), row.end());
            g.col.insert(g.col.end(), row.begin(), row.end());
            g.rp[i + 1] = (int32_t)g.col.size();
        }
    }
    const Csr& g = S.g;
    const int64_t nnzb = g.nnz();
    if (nnzb >= INT32_MAX) return "too many blocks for 32-bit indices";
    // column offsets from the row in 16 bits (half the index stream of the
    // finest-level products) when the node numbering keeps every neighbour
    // within 32767 of the node
    {
        bool fits = true;
        for (int i = 0; i < N && fits; ++i)
            for (int k = g.rp[i]; k < g.rp[i + 1]; ++k)
                if (g.col[k] - i > 32767 || g.col[k] - i < -32767) {
                    fits = false;
                    break;
                }
        S.dcol.clear();
        if (fits) {
            S.dcol.resize(nnzb);
            for (int i = 0; i < N; ++i)
                for (int k = g.rp[i]; k < g.rp[i + 1]; ++k) S.dcol[k] = (int16_t)(g.col[k] - i);
        }
        // fixed-width rows (no row-pointer load in the FP32 products) when no
        // row is longer than 16 blocks and the slots still have 32-bit indices
        int wmax = 0;
        for (int i = 0; i < N; ++i) wmax = std::max(wmax, g.rp[i + 1] - g.rp[i]);
        S.ell = (fits && wmax <= 16 && (int64_t)N * wmax <= INT32_MAX) ? wmax : 0;
        S.dcol_ell.clear();
        if (S.ell > 0) {
            S.dcol_ell.assign((size_t)N * S.ell, 0);
            for (int i = 0; i < N; ++i)
                for (int k = g.rp[i]; k < g.rp[i + 1]; ++k) S.dcol_ell[(size_t)i * S.ell + (k - g.rp[i])] = S.dcol[k];
        }
    }
    S.diag_pos.resize(N);
    S.row_of.resize(nnzb);
    S.tmap.resize(nnzb);
    for (int i = 0; i < N; ++i) {
        S.diag_pos[i] = (int32_t)find_in_row(g, i, i);
        for (int k = g.rp[i]; k < g.rp[i + 1]; ++k) {
            S.row_of[k] = i;
            S.tmap[k] = (int32_t)find_in_row(g, g.col[k], i);
        }
    }

    // element colouring; elements stored sorted by colour (stable)
    {
        std::vector<int32_t> col;
        int nc = greedy_colors(E, 4, m->h_tets, N, col);
        if (nc < 0) return "element colouring needs more than 256 colours";
        S.n_colors = nc;
        S.color_of = col;
        S.color_ptr.assign(nc + 1, 0);
        for (int e = 0; e < E; ++e) S.color_ptr[col[e] + 1]++;
        for (int c = 0; c < nc; ++c) S.color_ptr[c + 1] += S.color_ptr[c];
        std::vector<int32_t> fill(S.color_ptr.begin(), S.color_ptr.end() - 1);
        S.elem_perm.resize(E);
        for (int e = 0; e < E; ++e) S.elem_perm[fill[col[e]]++] = e;
        S.tets.resize((size_t)E * 4);
        S.emap.resize((size_t)E * 16);
        std::vector<int32_t> sorted_pos(E);
        for (int s = 0; s < E; ++s) {
            sorted_pos[S.elem_perm[s]] = s;
            const int32_t* t = m->h_tets + 4 * (size_t)S.elem_perm[s];
            for (int a = 0; a < 4; ++a) S.tets[4 * (size_t)s + a] = t[a];
        }
        // block index of (t[a], t[b]): positions of row t[a]'s columns, set
        // once per node, read by every element slot at that node
        std::vector<int32_t> pos(N, -1);
        for (int i = 0; i < N; ++i) {
            for (int k = g.rp[i]; k < g.rp[i + 1]; ++k) pos[g.col[k]] = k;
            for (int t = nptr[i]; t < nptr[i + 1]; ++t) {
                const int e = nelem[t] / 4, a = nelem[t] % 4;
                const int32_t* tet = m->h_tets + 4 * (size_t)e;
                for (int b = 0; b < 4; ++b) S.emap[16 * (size_t)sorted_pos[e] + 4 * a + b] = pos[tet[b]];
            }
        }
    }

    // outlets: slots = the distinct nodes of each outlet, ascending
    S.optr.assign(NO + 1, 0);
    S.slot_of.assign(N, -1);
    if (NO > 0) {
        S.F = m->h_outlet_ptr[NO];
        if (m->h_outlet_ptr[0] != 0) return "outlet_ptr[0] must be 0";
        for (int k = 0; k < NO; ++k)
            if (m->h_outlet_ptr[k + 1] < m->h_outlet_ptr[k]) return "outlet_ptr must be non-decreasing";
        for (int64_t f = 0; f < (int64_t)S.F * 3; ++f)
            if (m->h_faces[f] < 0 || m->h_faces[f] >= N) return "face vertex index out of range";
        std::vector<int32_t> face_out(S.F);
        for (int k = 0; k < NO; ++k) {
            std::set<int32_t> nodes;
            for (int f = m->h_outlet_ptr[k]; f < m->h_outlet_ptr[k + 1]; ++f) {
                face_out[f] = k;
                for (int a = 0; a < 3; ++a) nodes.insert(m->h_faces[3 * f + a]);
            }
            for (int32_t nd : nodes) {
                if (S.slot_of[nd] != -1) return "outlets share a node";
                S.slot_of[nd] = (int32_t)S.onode.size();
                S.onode.push_back(nd);
                S.oid.push_back(k);
            }
            S.optr[k + 1] = (int32_t)S.onode.size();
        }
        std::vector<int32_t> fc;
        int nfc = greedy_colors(S.F, 3, m->h_faces, N, fc);
        if (nfc < 0) return "face colouring needs more than 256 colours";
        S.n_fcolors = nfc;
        S.fcolor_ptr.assign(nfc + 1, 0);
        for (int f = 0; f < S.F; ++f) S.fcolor_ptr[fc[f] + 1]++;
        for (int c = 0; c < nfc; ++c) S.fcolor_ptr[c + 1] += S.fcolor_ptr[c];
        std::vector<int32_t> fill(S.fcolor_ptr.begin(), S.fcolor_ptr.end() - 1);
        std::vector<int32_t> perm(S.F);
        for (int f = 0; f < S.F; ++f) perm[fill[fc[f]]++] = f;
        S.faces.resize((size_t)S.F * 3);
        S.face_out.resize(S.F);
        S.fmap.resize((size_t)S.F * 9);
        S.fslot.resize((size_t)S.F * 3);
        for (int s = 0; s < S.F; ++s) {
            int f = perm[s];
            S.face_out[s] = face_out[f];
            for (int a = 0; a < 3; ++a) {
                int na = m->h_faces[3 * f + a];
                S.faces[3 * s + a] = na;
                S.fslot[3 * s + a] = S.slot_of[na];
                for (int b = 0; b < 3; ++b) {
                    int64_t q = find_in_row(g, na, m->h_faces[3 * f + b]);
                    if (q < 0) return "outlet face is not a face of the mesh";
                    S.fmap[9 * s + 3 * a + b] = (int32_t)q;
                }
            }
        }
    }

    // S_hat pattern: i ~ j when j is within distance 2 of i in the node graph
    {
        S.shat.n = N;
        S.shat.rp.assign(N + 1, 0);
        std::vector<int32_t> mark(N, -1), row;
        std::vector<int32_t> col;
        col.reserve((size_t)nnzb * 4);
        for (int i = 0; i < N; ++i) {
            row.clear();
            for (int k = g.rp[i]; k < g.rp[i + 1]; ++k) {
                int kk = g.col[k];
                for (int q = g.rp[kk]; q < g.rp[kk + 1]; ++q) {
                    int j = g.col[q];
                    if (mark[j] != i) {
                        mark[j] = i;
                        row.push_back(j);
                    }
                }
            }
            std::sort(row.begin(), row.end());
            col.insert(col.end(), row.begin(), row.end());
            S.shat.rp[i + 1] = (int32_t)col.size();
        }
        S.shat.col.swap(col);
    }

    // AMG hierarchy: levels of node aggregates (composed greedy matchings)
    {
        const int coarse_nodes = o.coarse_nodes > 0 ? o.coarse_nodes : 128;
        const int max_levels = o.max_levels > 0 ? o.max_levels : 16;
        const int coarse_matchings = o.coarse_matchings > 0 ? o.coarse_matchings : 3;
        if (coarse_matchings < 2 || coarse_matchings > 4) return "coarse_matchings must be in [2, 4]";
        S.lv.clear();
        S.lv.emplace_back();
        S.lv[0].n = N;
        S.lv[0].a = g;
        S.lv[0].s = S.shat;
        while (S.lv.back().n > coarse_nodes && (int)S.lv.size() < max_levels) {
            AmgLevelSym& f = S.lv.back();
            // compose k greedy matchings: node -> pair -> ... -> aggregate
            const int k = S.lv.size() == 1 ? 2 : coarse_matchings;
            std::vector<int32_t> agg(f.n);
            for (int i = 0; i < f.n; ++i) agg[i] = i;
            Csr cur = f.a;
            int n2 = f.n;
            for (int m = 0; m < k; ++m) {
                int nm = 0;
                std::vector<int32_t> am = greedy_matching(cur, nm);
                for (int i = 0; i < f.n; ++i) agg[i] = am[agg[i]];
                if (m + 1 < k) cur = quotient(cur, am, nm);
                n2 = nm;
            }
            if (n2 >= f.n) break;
            f.agg.swap(agg);
            f.aptr.assign(n2 + 1, 0);
            for (int i = 0; i < f.n; ++i) f.aptr[f.agg[i] + 1]++;
            for (int c = 0; c < n2; ++c) f.aptr[c + 1] += f.aptr[c];
            f.anodes.resize(f.n);
            std::vector<int32_t> fill(f.aptr.begin(), f.aptr.end() - 1);
            for (int i = 0; i < f.n; ++i) f.anodes[fill[f.agg[i]]++] = i;
            AmgLevelSym c;
            c.n = n2;
            c.a = quotient(f.a, f.agg, n2);
            c.s = quotient(f.s, f.agg, n2);
            gather_lists(f.a, c.a, f.agg, c.gptr, c.gidx);
            gather_lists(f.s, c.s, f.agg, c.sgptr, c.sgidx);
            c.a_qrow.resize(c.a.col.size());
            for (int I = 0; I < n2; ++I)
                for (int q = c.a.rp[I]; q < c.a.rp[I + 1]; ++q) c.a_qrow[q] = I;
            S.lv.push_back(std::move(c));
        }
    }
    return "";
}

}  // namespace ns

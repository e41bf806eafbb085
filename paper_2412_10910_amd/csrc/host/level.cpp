// Level setup: DoF numbering of continuous Q_k on an unstructured quad/hex
// mesh, the constrained set, device layouts and the setup kernels.
//
// Every local node of a cell belongs to one mesh entity (vertex, edge, face or
// cell interior).  Shared entities are identified by their global vertex ids,
// and their interior nodes are numbered in an orientation that every cell can
// reproduce from those ids alone:
//   edge: from the endpoint with the lower vertex id to the other one;
//   face: origin at the corner with the lowest id, first axis towards the
//         origin's face-neighbour corner with the lower id.
// DoFs are numbered entity by entity in order of first touch (cells in input
// order, local nodes lexicographic), which keeps the DoFs of neighbouring
// cells close in memory.
#include <algorithm>
#include <cstdint>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <unordered_map>

#include "../internal.hpp"

namespace nnmg {

namespace {

struct Key4Hash {
    size_t operator()(const std::array<int32_t, 4>& k) const {
        uint64_t h = 1469598103934665603ull;
        for (int32_t v : k) {
            h ^= (uint32_t)v;
            h *= 1099511628211ull;
        }
        return (size_t)h;
    }
};

inline uint64_t edge_key(int32_t a, int32_t b) {
    const uint32_t lo = (uint32_t)std::min(a, b), hi = (uint32_t)std::max(a, b);
    return ((uint64_t)lo << 32) | hi;
}

}  // namespace

void level_retain(Level* l) { l->refs.fetch_add(1); }

void level_reserve_rhs(Level& l, int nr) {
    if (nr < 1 || nr > kMaxRhs) fail(NNMG_ERR_INVALID_ARG, "number of right-hand sides must be in 1..8");
    if (nr <= l.contrib_rhs) return;
    NNMG_HIP(hipSetDevice(l.ctx->device));
    NNMG_HIP(hipDeviceSynchronize());  // earlier launches may still use the buffer
    l.d_contrib.alloc(l.ctx, std::max<size_t>(l.contrib_len * l.ncomp * (size_t)nr, 1) * sizeof(double));
    l.contrib_rhs = nr;
}

void level_release(Level* l) {
    if (l && l->refs.fetch_sub(1) == 1) delete static_cast<nnmg_level*>(l);
}

// Cell visiting order of the operator: blocks of cpb consecutive cells in
// input order (the x-runs whose shared faces the operator kernel merges), the
// blocks in Morton order of their centroids, so that the cells around a node
// are processed close in time (their contribution slots share cache lines,
// their source values L2 lines) and each XCD's contiguous range of blocks is
// a compact region.  NNMG_CELL_ORDER=input keeps the input order.
static std::vector<int64_t> cell_visit_order(const Level& L) {
    const int dim = L.dim, nvx = 1 << dim;
    const int64_t C = L.n_cells, cpb = L.cpb, nb = (C + cpb - 1) / cpb;
    std::vector<int64_t> bperm((size_t)nb);
    for (int64_t b = 0; b < nb; ++b) bperm[(size_t)b] = b;
    const char* ord = std::getenv("NNMG_CELL_ORDER");
    if (!(ord && std::string(ord) == "input") && nb > 1) {
        std::vector<double> cen((size_t)(nb * dim), 0.0);
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t c0 = b * cpb, c1 = std::min<int64_t>(C, c0 + cpb);
            for (int64_t c = c0; c < c1; ++c)
                for (int v = 0; v < nvx; ++v)
                    for (int a = 0; a < dim; ++a)
                        cen[(size_t)(b * dim + a)] += L.vertices[(size_t)(L.cells[(size_t)(c * nvx + v)] * dim + a)];
            for (int a = 0; a < dim; ++a) {
                cen[(size_t)(b * dim + a)] /= (double)((c1 - c0) * nvx);
                lo[a] = std::min(lo[a], cen[(size_t)(b * dim + a)]);
                hi[a] = std::max(hi[a], cen[(size_t)(b * dim + a)]);
            }
        }
        std::vector<uint64_t> code((size_t)nb, 0);
        for (int64_t b = 0; b < nb; ++b) {
            uint32_t qv[3] = {0, 0, 0};
            for (int a = 0; a < dim; ++a) {
                const double span = hi[a] - lo[a];
                const double t = span > 0 ? (cen[(size_t)(b * dim + a)] - lo[a]) / span : 0.0;
                qv[a] = (uint32_t)std::min(1023.0, std::max(0.0, std::floor(t * 1024.0)));
            }
            uint64_t m = 0;
            for (int bit = 9; bit >= 0; --bit)
                for (int a = dim - 1; a >= 0; --a) m = (m << 1) | ((qv[a] >> bit) & 1u);
            code[(size_t)b] = m;
        }
        std::stable_sort(bperm.begin(), bperm.end(),
                         [&](int64_t x, int64_t y) { return code[(size_t)x] < code[(size_t)y]; });
    }
    std::vector<int64_t> visit;
    visit.reserve((size_t)C);
    for (int64_t b : bperm)
        for (int64_t c = b * cpb; c < std::min<int64_t>(C, (b + 1) * cpb); ++c) visit.push_back(c);
    return visit;
}

static void number_dofs(Level& L, const std::vector<int64_t>& visit) {
    const int dim = L.dim, k = L.degree, n = L.n, q = L.q, nv = 1 << dim;
    const int64_t C = L.n_cells;
    const int64_t V = (int64_t)L.vertices.size() / dim;
    const int32_t* cells = L.cells.data();

    std::vector<int64_t> vertex_base(V, -1);
    std::unordered_map<uint64_t, int64_t> edge_base;
    std::unordered_map<std::array<int32_t, 4>, int64_t, Key4Hash> face_base;
    edge_base.reserve((size_t)(C * (dim == 3 ? 3 : 2) + 16));
    if (dim == 3) face_base.reserve((size_t)(C * 3 + 16));
    int64_t next = 0;
    const int ke = k - 1;  // interior nodes per edge direction

    L.dofmap.assign((size_t)(C * q), -1);
    // per cell, the base of each edge and face met so far and its orientation
    // (entity e = cx + 3 cy + 9 cz of the node classes 0 / inside / k): one
    // lookup per entity instead of one per node, the same first-touch order
    int64_t ebase[27];
    int eflip[27];
    for (int64_t vi = 0; vi < C; ++vi) {
        const int64_t c = visit[(size_t)vi];
        const int32_t* cv = cells + c * nv;
        int64_t interior_base = -1;
        for (int e = 0; e < 27; ++e) ebase[e] = -1;
        for (int a = 0; a < q; ++a) {
            int id[3] = {a % n, (a / n) % n, dim == 3 ? a / (n * n) : 0};
            int n_int = 0, int_axes[3];
            for (int d = 0; d < dim; ++d)
                if (id[d] > 0 && id[d] < k) int_axes[n_int++] = d;
            int ent = 0;
            for (int d = dim - 1; d >= 0; --d) ent = 3 * ent + (id[d] == 0 ? 0 : (id[d] == k ? 2 : 1));
            int64_t dof;
            if (n_int == 0) {
                int b = 0;
                for (int d = 0; d < dim; ++d) b |= (id[d] == k ? 1 : 0) << d;
                const int32_t v = cv[b];
                if (vertex_base[v] < 0) vertex_base[v] = next++;
                dof = vertex_base[v];
            } else if (n_int == 1 && n_int < dim) {
                const int ax = int_axes[0];
                if (ebase[ent] < 0) {
                    int b0 = 0;
                    for (int d = 0; d < dim; ++d)
                        if (d != ax) b0 |= (id[d] == k ? 1 : 0) << d;
                    const int32_t v0 = cv[b0], v1 = cv[b0 | (1 << ax)];
                    const uint64_t key = edge_key(v0, v1);
                    auto it = edge_base.find(key);
                    if (it == edge_base.end()) {
                        ebase[ent] = next;
                        next += ke;
                        edge_base.emplace(key, ebase[ent]);
                    } else {
                        ebase[ent] = it->second;
                    }
                    eflip[ent] = v0 < v1 ? 0 : 1;
                }
                const int t = id[ax];
                const int pos = eflip[ent] == 0 ? t - 1 : k - t - 1;
                dof = ebase[ent] + pos;
            } else if (n_int == 2 && dim == 3) {
                const int a0 = int_axes[0], a1 = int_axes[1];
                if (ebase[ent] < 0) {
                    int fixed = 3 - a0 - a1;
                    const int bf = (id[fixed] == k ? 1 : 0) << fixed;
                    auto corner = [&](int s, int t) { return cv[bf | (s << a0) | (t << a1)]; };
                    const int32_t c00 = corner(0, 0), c10 = corner(1, 0), c01 = corner(0, 1), c11 = corner(1, 1);
                    std::array<int32_t, 4> key{c00, c10, c01, c11};
                    std::sort(key.begin(), key.end());
                    auto it = face_base.find(key);
                    if (it == face_base.end()) {
                        ebase[ent] = next;
                        next += (int64_t)ke * ke;
                        face_base.emplace(key, ebase[ent]);
                    } else {
                        ebase[ent] = it->second;
                    }
                    // origin corner: lowest vertex id
                    int os = 0, ot = 0;
                    int32_t best = c00;
                    if (c10 < best) { best = c10; os = 1; ot = 0; }
                    if (c01 < best) { best = c01; os = 0; ot = 1; }
                    if (c11 < best) { best = c11; os = 1; ot = 1; }
                    const int32_t nb_s = corner(1 - os, ot);  // neighbour along axis a0
                    const int32_t nb_t = corner(os, 1 - ot);  // neighbour along axis a1
                    eflip[ent] = os | (ot << 1) | ((nb_s < nb_t ? 0 : 1) << 2);
                }
                const int os = eflip[ent] & 1, ot = (eflip[ent] >> 1) & 1;
                const int ds = os == 0 ? id[a0] : k - id[a0];
                const int dt = ot == 0 ? id[a1] : k - id[a1];
                int u, w;
                if (((eflip[ent] >> 2) & 1) == 0) {
                    u = ds;
                    w = dt;
                } else {
                    u = dt;
                    w = ds;
                }
                dof = ebase[ent] + (u - 1) + (int64_t)(w - 1) * ke;
            } else {
                // cell interior: the block is reserved when its first node is met
                if (interior_base < 0) {
                    interior_base = next;
                    int64_t cnt = 1;
                    for (int d = 0; d < dim; ++d) cnt *= ke;
                    next += cnt;
                }
                int64_t pos = 0, stride = 1;
                for (int d = 0; d < dim; ++d) {
                    pos += (id[d] - 1) * stride;
                    stride *= ke;
                }
                dof = interior_base + pos;
            }
            L.dofmap[(size_t)(c * q + a)] = (int32_t)dof;
        }
    }
    if (next > INT32_MAX) fail(NNMG_ERR_UNSUPPORTED, "more than 2^31 DoFs");
    L.n_nodes = next;
}

// Entity-compressed operator indices (layout in Level::d_ent_rec).  The DoFs
// of every mesh entity are contiguous in a canonical orientation (see
// number_dofs), so a cell needs one DoF base and one orientation code per
// entity instead of one index per local node.  The orientation is found by
// trying the codes against the cell's DoF map, so the record reproduces the
// map exactly whatever the numbering rule.  The x-face between consecutive
// cells of a block is merged (summed in the kernel before the store) where
// every line of the two cells meets on it, and the slots are laid out
// DoF-major with one slot per writing cell in visiting order, so the slot
// offsets stay sorted by DoF and every sum keeps a fixed order.  Returns
// false, leaving the level on the per-node layout, where the mesh does not fit
// the record: an entity with constrained and unconstrained nodes, no code
// reproducing the map, or more than 15 writers of one entity.
static bool build_entity_records(const Level& L, std::vector<int32_t>& rec, std::vector<int32_t>& off) {
    const int n = L.n, k = L.degree, ke = k - 1, q = L.q, cpb = L.cpb;
    struct Node {
        int a, u, v, w;
    };
    std::vector<Node> nodes[27];
    int edim[27] = {};
    for (int a = 0; a < q; ++a) {
        const int id[3] = {a % n, (a / n) % n, a / (n * n)};
        int cls[3], loc[3] = {0, 0, 0}, m = 0;
        for (int d = 0; d < 3; ++d) {
            cls[d] = id[d] == 0 ? 0 : (id[d] == k ? 2 : 1);
            if (cls[d] == 1) loc[m++] = id[d] - 1;
        }
        const int e = cls[0] + 3 * cls[1] + 9 * cls[2];
        nodes[e].push_back({a, loc[0], loc[1], loc[2]});
        edim[e] = m;
    }
    auto canon = [&](const Node& nd, int o) {
        int u = (o & 1) ? ke - 1 - nd.u : nd.u;
        int v = (o & 2) ? ke - 1 - nd.v : nd.v;
        if (o & 4) std::swap(u, v);
        return u + ke * (v + ke * nd.w);
    };
    const int64_t P = L.nblocks * cpb;
    std::vector<int32_t> base((size_t)(P * 27), -1), rank((size_t)(P * 27), -1);
    std::vector<uint8_t> orient((size_t)(P * 27), 0), flags((size_t)P, 0);
    std::vector<int32_t> ndof_at((size_t)L.n_nodes, 0);
    for (int64_t p = 0; p < P; ++p) {
        const int64_t c = L.order[(size_t)p];
        if (c < 0) continue;
        const int32_t* dm = &L.dofmap[(size_t)(c * q)];
        for (int e = 0; e < 27; ++e) {
            int32_t b = INT32_MAX;
            int ncons = 0;
            for (const Node& nd : nodes[e]) {
                b = std::min(b, dm[nd.a]);
                ncons += L.constrained[(size_t)dm[nd.a]];
            }
            if (ncons != 0 && ncons != (int)nodes[e].size()) return false;
            const int no = edim[e] == 1 ? 2 : (edim[e] == 2 ? 8 : 1);
            int found = -1;
            for (int o = 0; o < no && found < 0; ++o) {
                bool same = true;
                for (const Node& nd : nodes[e])
                    if (dm[nd.a] != b + canon(nd, o)) {
                        same = false;
                        break;
                    }
                if (same) found = o;
            }
            if (found < 0) return false;
            base[(size_t)(p * 27 + e)] = b;
            orient[(size_t)(p * 27 + e)] = (uint8_t)found;
            ndof_at[(size_t)b] = (int32_t)nodes[e].size();
        }
        // merge with the previous cell of the block across a shared x-face
        if (p % cpb > 0 && L.order[(size_t)(p - 1)] >= 0) {
            const int32_t* dp = &L.dofmap[(size_t)(L.order[(size_t)(p - 1)] * q)];
            bool same = true;
            for (int line = 0; line < n * n && same; ++line) same = dp[k + n * line] == dm[n * line];
            if (same) {
                flags[(size_t)(p - 1)] |= 2;
                flags[(size_t)p] |= 1;
            }
        }
    }
    // writers of every entity, ranked in visiting order
    std::vector<int32_t> cnt((size_t)L.n_nodes, 0);
    for (int64_t p = 0; p < P; ++p) {
        if (L.order[(size_t)p] < 0) continue;
        for (int e = 0; e < 27; ++e) {
            const int32_t b = base[(size_t)(p * 27 + e)];
            if (L.constrained[(size_t)b]) continue;
            if (e % 3 == 0 && (flags[(size_t)p] & 1)) continue;  // added by the previous cell
            rank[(size_t)(p * 27 + e)] = cnt[(size_t)b]++;
            if (cnt[(size_t)b] > 15) return false;
        }
    }
    off.assign((size_t)L.n_nodes + 1, 0);
    int64_t cur = 0;
    for (int64_t d = 0; d < L.n_nodes;) {
        const int nd = ndof_at[(size_t)d];
        if (nd <= 0) return false;  // not the first DoF of an entity: numbering not entity-contiguous
        const int c = L.constrained[(size_t)d] ? 0 : cnt[(size_t)d];
        for (int t = 0; t < nd; ++t) off[(size_t)(d + t)] = (int32_t)(cur + (int64_t)t * c);
        cur += (int64_t)nd * c;
        if (cur >= (int64_t)kMergeNext) return false;
        d += nd;
    }
    off[(size_t)L.n_nodes] = (int32_t)cur;
    rec.assign((size_t)(L.nblocks * kEntWords * cpb), 0);
    for (int64_t p = 0; p < P; ++p) {
        const int64_t blk = p / cpb, cell = p % cpb;
        auto W = [&](int w) -> int32_t& { return rec[(size_t)((blk * kEntWords + w) * cpb + cell)]; };
        if (L.order[(size_t)p] < 0) {
            for (int e = 0; e < 27; ++e) W(e) = W(27 + e) = -1;
            continue;
        }
        for (int e = 0; e < 27; ++e) {
            const int32_t b = base[(size_t)(p * 27 + e)];
            const bool cons = L.constrained[(size_t)b] != 0;
            const int32_t r = rank[(size_t)(p * 27 + e)];
            W(e) = cons ? -1 : b;
            W(27 + e) = (cons || r < 0) ? -1 : off[(size_t)b] + r;
            const int32_t code = (cons ? 0 : cnt[(size_t)b]) | (orient[(size_t)(p * 27 + e)] << 4);
            W(54 + e / 4) |= code << (8 * (e % 4));
        }
        W(61) = flags[(size_t)p];
    }
    return true;
}

static void find_constraints(Level& L, const uint8_t* dirichlet) {
    const int dim = L.dim, k = L.degree, n = L.n, q = L.q, nv = 1 << dim;
    const int64_t C = L.n_cells;
    L.constrained.assign((size_t)L.n_nodes, 0);
    if (!dirichlet) return;
    const int fv = 1 << (dim - 1);
    std::unordered_map<std::array<int32_t, 4>, int, Key4Hash> count;
    auto facet_key = [&](int64_t c, int ax, int side) {
        std::array<int32_t, 4> key{-1, -1, -1, -1};
        int m = 0;
        for (int b = 0; b < nv; ++b)
            if (((b >> ax) & 1) == side) key[m++] = L.cells[(size_t)(c * nv + b)];
        std::sort(key.begin(), key.begin() + fv);
        return key;
    };
    // only a facet whose vertices are all Dirichlet-marked can be constrained,
    // and every cell holding such a facet sees the same vertices: counting
    // those facets alone tells which of them lie on the boundary
    auto all_marked = [&](int64_t c, int ax, int side) {
        for (int b = 0; b < nv; ++b)
            if (((b >> ax) & 1) == side && !dirichlet[L.cells[(size_t)(c * nv + b)]]) return false;
        return true;
    };
    for (int64_t c = 0; c < C; ++c)
        for (int ax = 0; ax < dim; ++ax)
            for (int side = 0; side < 2; ++side)
                if (all_marked(c, ax, side)) count[facet_key(c, ax, side)]++;
    for (int64_t c = 0; c < C; ++c)
        for (int ax = 0; ax < dim; ++ax)
            for (int side = 0; side < 2; ++side) {
                if (!all_marked(c, ax, side)) continue;
                const auto key = facet_key(c, ax, side);
                if (count[key] != 1) continue;
                for (int a = 0; a < q; ++a) {
                    const int id = ax == 0 ? a % n : (ax == 1 ? (a / n) % n : a / (n * n));
                    if (id == side * k) L.constrained[(size_t)L.dofmap[(size_t)(c * q + a)]] = 1;
                }
            }
}

static void compute_support_points(Level& L) {
    const int dim = L.dim, n = L.n, q = L.q, nv = 1 << dim;
    L.support.assign((size_t)(L.n_nodes * dim), 0.0);
    std::vector<char> done((size_t)L.n_nodes, 0);
    // the trilinear weights of the vertices at each local node (the same
    // products, in the same order, for every cell)
    std::vector<double> W((size_t)(q * nv));
    for (int a = 0; a < q; ++a) {
        const double xi[3] = {L.basis.node[a % n], L.basis.node[(a / n) % n],
                              dim == 3 ? L.basis.node[a / (n * n)] : 0.0};
        for (int b = 0; b < nv; ++b) {
            double N = 1.0;
            for (int d = 0; d < dim; ++d) N *= ((b >> d) & 1) ? xi[d] : 1.0 - xi[d];
            W[(size_t)(a * nv + b)] = N;
        }
    }
    // each DoF takes the coordinates its first cell gives it
    for (int64_t c = 0; c < L.n_cells; ++c) {
        const int32_t* cv = &L.cells[(size_t)(c * nv)];
        for (int a = 0; a < q; ++a) {
            const int32_t dof = L.dofmap[(size_t)(c * q + a)];
            if (done[(size_t)dof]) continue;
            done[(size_t)dof] = 1;
            const double* w = &W[(size_t)(a * nv)];
            for (int i = 0; i < dim; ++i) {
                double x = 0.0;
                for (int b = 0; b < nv; ++b) x += w[b] * L.vertices[(size_t)(cv[b] * dim + i)];
                L.support[(size_t)(dof * dim + i)] = x;
            }
        }
    }
}

Level* level_create(Ctx* ctx, const nnmg_mesh* mesh, int degree, const nnmg_level_opts& opts) {
    if (!mesh) fail(NNMG_ERR_INVALID_ARG, "mesh is NULL");
    if (opts.op != NNMG_OP_LAPLACE && opts.op != NNMG_OP_ELASTICITY) fail(NNMG_ERR_INVALID_ARG, "operator");
    if (opts.op == NNMG_OP_ELASTICITY) {
        if (mesh->dim != 3) fail(NNMG_ERR_UNSUPPORTED, "the elasticity operator is three-dimensional");
        if (!(opts.mu > 0.0) || !(opts.lambda >= 0.0) || !std::isfinite(opts.lambda) || !std::isfinite(opts.mu))
            fail(NNMG_ERR_INVALID_ARG, "Lame coefficients must satisfy mu > 0, lambda >= 0");
    }
    if (mesh->dim != 2 && mesh->dim != 3) fail(NNMG_ERR_UNSUPPORTED, "dim must be 2 or 3");
    if (degree < 1 || degree > 4) fail(NNMG_ERR_UNSUPPORTED, "degree must be in 1..4");
    if (mesh->n_vertices <= 0 || mesh->n_cells <= 0 || !mesh->vertices || !mesh->cells)
        fail(NNMG_ERR_INVALID_ARG, "empty mesh");
    if (mesh->n_vertices > INT32_MAX || mesh->n_cells > INT32_MAX / 125)
        fail(NNMG_ERR_UNSUPPORTED, "mesh too large for 32-bit indices");
    const int dim = mesh->dim, nv = 1 << dim;
    for (int64_t i = 0; i < mesh->n_vertices * dim; ++i)
        if (!std::isfinite(mesh->vertices[i])) fail(NNMG_ERR_MESH, "non-finite vertex coordinate");
    for (int64_t c = 0; c < mesh->n_cells; ++c) {
        for (int b = 0; b < nv; ++b) {
            const int32_t v = mesh->cells[c * nv + b];
            if (v < 0 || v >= mesh->n_vertices) fail(NNMG_ERR_MESH, "cell vertex index out of range");
            for (int b2 = 0; b2 < b; ++b2)
                if (mesh->cells[c * nv + b2] == v) fail(NNMG_ERR_MESH, "repeated vertex in a cell");
        }
    }

    auto* L = new nnmg_level();
    try {
        L->ctx = ctx;
        L->dim = dim;
        L->degree = degree;
        L->n = degree + 1;
        L->q = dim == 3 ? L->n * L->n * L->n : L->n * L->n;
        vmult_shape(dim, L->n, &L->wg, &L->cpb);
        L->n_cells = mesh->n_cells;
        L->basis = make_basis(degree);
        L->vertices.assign(mesh->vertices, mesh->vertices + mesh->n_vertices * dim);
        L->cells.assign(mesh->cells, mesh->cells + mesh->n_cells * nv);

        L->op = opts.op;
        L->ncomp = opts.op == NNMG_OP_ELASTICITY ? dim : 1;
        L->lam = opts.lambda;
        L->mu = opts.mu;
        // DoFs by first touch in input order (measured: numbering them in the
        // blocks' Morton order made the transfers slower and cancelled the
        // operator's gain from processing the blocks in that order)
        std::vector<int64_t> input_order((size_t)L->n_cells);
        for (int64_t c = 0; c < L->n_cells; ++c) input_order[(size_t)c] = c;
        number_dofs(*L, input_order);
        const std::vector<int64_t> visit = cell_visit_order(*L);
        find_constraints(*L, mesh->dirichlet_vertex);
        compute_support_points(*L);
        if (L->n_nodes * L->ncomp > INT32_MAX) fail(NNMG_ERR_UNSUPPORTED, "more than 2^31 DoFs");
        L->n_dofs = L->n_nodes * L->ncomp;
        for (int64_t i = 0; i < L->n_nodes; ++i)
            if (L->constrained[(size_t)i])
                for (int c = 0; c < L->ncomp; ++c) L->constrained_idx.push_back((int32_t)(i * L->ncomp + c));
        L->n_free = L->n_dofs - (int64_t)L->constrained_idx.size();

        NNMG_HIP(hipSetDevice(ctx->device));
        // device cell->DoF maps, constrained DoFs encoded as -1
        const int q = L->q, n = L->n, M = dim * (dim + 1) / 2;
        std::vector<int32_t> enc(L->dofmap.size());
        for (size_t i = 0; i < enc.size(); ++i) enc[i] = L->constrained[(size_t)L->dofmap[i]] ? -1 : L->dofmap[i];
        L->d_dofmap.upload(ctx, enc);
        // block positions: the cells in visiting order (blocks of cpb input-order
        // cells, the blocks in Morton order; see cell_visit_order), the last
        // block padded
        L->nblocks = (L->n_cells + L->cpb - 1) / L->cpb;
        L->order.assign((size_t)(L->nblocks * L->cpb), -1);
        {
            int64_t p = 0;
            for (int64_t i = 0; i < L->n_cells; ++i) {
                const int64_t c = visit[(size_t)i];
                // a padded (short) block keeps its own positions
                if (i > 0 && c / L->cpb != visit[(size_t)(i - 1)] / L->cpb) p = ((p + L->cpb - 1) / L->cpb) * L->cpb;
                L->order[(size_t)p++] = (int32_t)c;
            }
        }
        L->d_order.upload(ctx, L->order);
        // operator layout: lane (cell_in_block, line) holds the x-line `line` of its cell
        const int Lc = dim == 3 ? n * n : n, WG = L->wg;
        std::vector<int32_t> blk((size_t)(L->nblocks * n * WG), -1);
        for (int64_t p = 0; p < L->nblocks * L->cpb; ++p) {
            const int64_t c = L->order[(size_t)p];
            if (c < 0) continue;
            const int64_t b = p / L->cpb;
            const int cell = (int)(p - b * L->cpb);
            for (int a = 0; a < q; ++a) {
                const int i = a % n, line = a / n;
                blk[(size_t)((b * n + i) * WG + cell * Lc + line)] = enc[(size_t)(c * q + a)];
            }
        }
        L->d_dofmap_blk.upload(ctx, blk);
        // contribution slots: the (cell, node) contributions of DoF i occupy
        // [off[i], off[i+1]) of a DoF-sorted buffer; pos_blk gives each lane's slots.
        // Where the first node of a lane's x-line is the same DoF as the last
        // node of the same line of the previous cell in the block (and both
        // lanes are in one wavefront), the kernel adds the two in registers:
        // the first node gets no slot and the last node's slot carries
        // kMergeNext.
        {
            std::vector<uint8_t> merged(blk.size(), 0), receives(blk.size(), 0);
            for (int64_t b = 0; b < L->nblocks; ++b)
                for (int p = 1; p < L->cpb; ++p)
                    for (int line = 0; line < Lc; ++line) {
                        const int lane0 = p * Lc + line, laneL = (p - 1) * Lc + line;
                        if (lane0 / kWaveLanes != laneL / kWaveLanes) continue;
                        const size_t k0 = (size_t)((b * n + 0) * WG + lane0);
                        const size_t kL = (size_t)((b * n + (n - 1)) * WG + laneL);
                        if (blk[k0] >= 0 && blk[k0] == blk[kL]) {
                            merged[k0] = 1;
                            receives[kL] = 1;
                        }
                    }
            std::vector<int32_t> off((size_t)L->n_nodes + 1, 0);
            for (size_t k = 0; k < blk.size(); ++k)
                if (blk[k] >= 0 && !merged[k]) off[(size_t)blk[k] + 1]++;
            for (int64_t i = 0; i < L->n_nodes; ++i) off[(size_t)i + 1] += off[(size_t)i];
            if ((int64_t)off[(size_t)L->n_nodes] * L->ncomp >= (int64_t)kMergeNext)
                fail(NNMG_ERR_UNSUPPORTED, "too many contributions");
            std::vector<int32_t> cur(off.begin(), off.end() - 1);
            std::vector<int32_t> pos(blk.size(), -1);
            for (size_t k = 0; k < blk.size(); ++k)
                if (blk[k] >= 0 && !merged[k]) pos[k] = cur[(size_t)blk[k]]++ | (receives[k] ? kMergeNext : 0);
            L->d_inv_off.upload(ctx, off);
            L->d_pos_blk.upload(ctx, pos);
            L->contrib_len = (size_t)off[(size_t)L->n_nodes];
        }
        // the entity-compressed indices of the same operator (3D Laplace,
        // degree >= 3, where a cell has far more nodes than entities)
        if (dim == 3 && L->op == NNMG_OP_LAPLACE && degree >= 3) {
            std::vector<int32_t> rec, off2;
            if (build_entity_records(*L, rec, off2)) {
                L->d_ent_rec.upload(ctx, rec);
                L->d_inv_off_ent.upload(ctx, off2);
                L->contrib_len = std::max(L->contrib_len, (size_t)off2[(size_t)L->n_nodes]);
                const char* ix = std::getenv("NNMG_INDEX");
                if (ix && std::string(ix) == "entity") L->var[0].index_layout = L->var[1].index_layout = 1;
            }
        }
        // ncomp values per slot: component c of slot k at ncomp * k + c (sized
        // for the larger of the two index layouts)
        L->d_contrib.alloc(ctx, std::max<size_t>(L->contrib_len * L->ncomp, 1) * sizeof(double));
        L->d_constrained.upload(ctx, L->constrained_idx);
        std::vector<double> cv((size_t)(L->n_cells * nv * dim));
        for (int64_t c = 0; c < L->n_cells; ++c)
            for (int b = 0; b < nv; ++b)
                for (int i = 0; i < dim; ++i)
                    cv[(size_t)((c * nv + b) * dim + i)] = L->vertices[(size_t)(L->cells[(size_t)(c * nv + b)] * dim + i)];
        L->d_cellverts.upload(ctx, cv);

        const size_t mlen = (size_t)(L->nblocks * M * n * WG);
        L->d_metric64.alloc(ctx, mlen);
        L->d_metric32.alloc(ctx, mlen);
        NNMG_HIP(hipMemset(L->d_metric64.ptr, 0, L->d_metric64.bytes()));
        NNMG_HIP(hipMemset(L->d_metric32.ptr, 0, L->d_metric32.bytes()));
        DeviceArray<int> bad;
        bad.alloc(ctx, 1);
        NNMG_HIP(hipMemset(bad.ptr, 0, sizeof(int)));
        launch_geometry(*L, bad.ptr, nullptr);
        int hbad = 0;
        NNMG_HIP(hipMemcpy(&hbad, bad.ptr, sizeof(int), hipMemcpyDeviceToHost));
        if (hbad) fail(NNMG_ERR_MESH, "cell with non-positive Jacobian determinant at a Gauss point");

        L->d_diag64.alloc(ctx, (size_t)L->n_dofs);
        NNMG_HIP(hipMemset(L->d_diag64.ptr, 0, L->d_diag64.bytes()));
        launch_diagonal(*L, L->d_diag64.ptr, nullptr);
        L->d_dinv64.alloc(ctx, (size_t)L->n_dofs);
        L->d_dinv32.alloc(ctx, (size_t)L->n_dofs);
        launch_invert_diagonal(*L, L->d_diag64.ptr, nullptr);
        launch_set_constrained(L->d_constrained.ptr, L->constrained_idx.size(), 1.0, L->d_diag64.ptr, NNMG_FP64,
                               nullptr);

        // coefficients of the Q1 map per cell, for the operator kernel that
        // rebuilds the geometry at the Gauss points
        const int NC = dim == 3 ? 21 : 6;
        std::vector<double> coef((size_t)(L->nblocks * NC * L->cpb), 0.0);
        for (int64_t p = 0; p < L->nblocks * L->cpb; ++p) {
            const int64_t b = p / L->cpb;
            const int cell = (int)(p - b * L->cpb);
            const int64_t c = L->order[(size_t)p];
            double X[8][3] = {};
            if (c >= 0) {
                for (int v = 0; v < nv; ++v)
                    for (int i = 0; i < dim; ++i) X[v][i] = cv[(size_t)((c * nv + v) * dim + i)];
            } else {
                // padding: the unit cell, so that the unused lanes see det J = 1
                for (int v = 0; v < nv; ++v)
                    for (int i = 0; i < dim; ++i) X[v][i] = (v >> i) & 1;
            }
            double vals[21];
            if (dim == 3) {
                for (int i = 0; i < 3; ++i) {
                    vals[0 + i] = X[1][i] - X[0][i];                                                // b
                    vals[3 + i] = X[2][i] - X[0][i];                                                // c
                    vals[6 + i] = X[4][i] - X[0][i];                                                // d
                    vals[9 + i] = X[3][i] - X[1][i] - X[2][i] + X[0][i];                            // e
                    vals[12 + i] = X[5][i] - X[1][i] - X[4][i] + X[0][i];                           // f
                    vals[15 + i] = X[6][i] - X[2][i] - X[4][i] + X[0][i];                           // g
                    vals[18 + i] = X[7][i] - X[3][i] - X[5][i] - X[6][i] + X[1][i] + X[2][i] + X[4][i] - X[0][i];  // h
                }
            } else {
                for (int i = 0; i < 2; ++i) {
                    vals[0 + i] = X[1][i] - X[0][i];                      // b
                    vals[2 + i] = X[2][i] - X[0][i];                      // c
                    vals[4 + i] = X[3][i] - X[1][i] - X[2][i] + X[0][i];  // d
                }
            }
            for (int m = 0; m < NC; ++m) coef[(size_t)((b * NC + m) * L->cpb + cell)] = vals[m];
        }
        L->d_coef64.upload(ctx, coef);
        std::vector<float> coef32(coef.begin(), coef.end());
        L->d_coef32.upload(ctx, coef32);
        const char* mode = std::getenv("NNMG_GEOMETRY");
        // the elasticity operator rebuilds J from the map coefficients
        const char* scatter = std::getenv("NNMG_SCATTER");
        const char* sweep = std::getenv("NNMG_SWEEP");
        for (auto& vr : L->var) {
            vr.sweep = sweep && std::string(sweep) == "transposed" && L->op == NNMG_OP_LAPLACE ? 1 : 0;
            vr.geometry_mode = (mode && std::string(mode) == "metric" && L->op == NNMG_OP_LAPLACE) ? 0 : 1;
            vr.atomic = scatter && std::string(scatter) == "atomic" && L->op == NNMG_OP_LAPLACE;
            if (vr.atomic) vr.index_layout = 0;
        }
        if (L->var[0].geometry_mode == 1) {
            NNMG_HIP(hipDeviceSynchronize());
            L->d_metric64.reset();
            L->d_metric32.reset();
        }
        NNMG_HIP(hipDeviceSynchronize());
    } catch (...) {
        delete L;
        throw;
    }
    return L;
}

void level_diagonal(const Level& L, int prec, void* out, hipStream_t s) {
    // the diagonal is assembled once at setup (1 on constrained rows)
    if (prec == NNMG_FP64)
        NNMG_HIP(hipMemcpyAsync(out, L.d_diag64.ptr, L.d_diag64.bytes(), hipMemcpyDeviceToDevice, s));
    else
        launch_cast_64_to_32(L.d_diag64.ptr, (float*)out, (size_t)L.n_dofs, s);
}

void level_quadrature_points(const Level& L, double* out) {
    const int dim = L.dim, n = L.n, q = L.q, nv = 1 << dim;
    for (int64_t c = 0; c < L.n_cells; ++c) {
        const int32_t* cv = &L.cells[(size_t)(c * nv)];
        for (int a = 0; a < q; ++a) {
            double xi[3] = {L.basis.gauss[a % n], L.basis.gauss[(a / n) % n], dim == 3 ? L.basis.gauss[a / (n * n)] : 0.0};
            for (int i = 0; i < dim; ++i) {
                double x = 0.0;
                for (int b = 0; b < nv; ++b) {
                    double N = 1.0;
                    for (int d = 0; d < dim; ++d) N *= ((b >> d) & 1) ? xi[d] : 1.0 - xi[d];
                    x += N * L.vertices[(size_t)(cv[b] * dim + i)];
                }
                out[(size_t)((c * q + a) * dim + i)] = x;
            }
        }
    }
}

}  // namespace nnmg

// Host construction of the per-mesh assembly plan (the global assembly step of Algorithm 2,
// where the sparsity pattern is fixed once per mesh).
//   1. node -> element lists (counting sort; ascending element id per node);
//   2. CSR pattern: row i holds every j that shares an element with i
//      (Section 3, step 2: compact support), sorted, structural zeros kept;
//   3. the element-entry -> CSR-slot permutation for the distinct symmetric
//      pairs of every element (upper-triangle slot), and the mirror map
//      (i,j) -> (j,i); the tile plan turns these into the fixed summation
//      order of the scatter.
#include <algorithm>
#include <thread>

#include "qxa_internal.hpp"

namespace qxa {


qxa_status build_host_plan(int dim, int order, int64_t n_nodes, int64_t n_elem, const int32_t *conn, HostPlan &hp)
{
    const int np = n_local(dim, order);
    const int ns = n_sym(np);
    if (uint64_t(ns) * uint64_t(n_elem) >= (uint64_t(1) << 32))
        return fail(QXA_E_UNSUPPORTED, "mesh too large for 32-bit element-entry indices");
    hp.n_nodes = n_nodes;
    hp.n_elem = n_elem;
    // 1. node -> element adjacency (the order within a node does not matter:
    //    each row's columns are sorted below)
    std::vector<int64_t> astart(n_nodes + 1, 0);
    parallel_for(n_elem, [&](int64_t lo, int64_t hi) {
        for (int i = 0; i < np; ++i)
            for (int64_t e = lo; e < hi; ++e) __atomic_fetch_add(&astart[conn[size_t(i) * n_elem + e] + 1], 1, __ATOMIC_RELAXED);
    });
    for (int64_t v = 0; v < n_nodes; ++v) astart[v + 1] += astart[v];
    hvec<int32_t> aelem(astart[n_nodes]);
    {
        std::vector<int64_t> fill(astart.begin(), astart.end() - 1);
        parallel_for(n_elem, [&](int64_t lo, int64_t hi) {
            for (int64_t e = lo; e < hi; ++e)
                for (int i = 0; i < np; ++i)
                    aelem[__atomic_fetch_add(&fill[conn[size_t(i) * n_elem + e]], 1, __ATOMIC_RELAXED)] = int32_t(e);
        });
    }
    // 2. pattern: count, then fill
    hp.row_ptr.assign(n_nodes + 1, 0);
    auto row_cols = [&](int64_t v, std::vector<int32_t> &buf) {
        buf.clear();
        for (int64_t p = astart[v]; p < astart[v + 1]; ++p) {
            const int64_t e = aelem[p];
            for (int j = 0; j < np; ++j) buf.push_back(conn[size_t(j) * n_elem + e]);
        }
        std::sort(buf.begin(), buf.end());
        buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
    };
    parallel_for(n_nodes, [&](int64_t lo, int64_t hi) {
        std::vector<int32_t> buf;
        for (int64_t v = lo; v < hi; ++v) {
            row_cols(v, buf);
            hp.row_ptr[v + 1] = int64_t(buf.size());
        }
    });
    for (int64_t v = 0; v < n_nodes; ++v) hp.row_ptr[v + 1] += hp.row_ptr[v];
    hp.nnz = hp.row_ptr[n_nodes];
    if (hp.nnz >= (int64_t(1) << 31)) return fail(QXA_E_UNSUPPORTED, "more than 2^31 nonzeros");
    hp.col_idx.resize(hp.nnz);
    parallel_for(n_nodes, [&](int64_t lo, int64_t hi) {
        std::vector<int32_t> buf;
        for (int64_t v = lo; v < hi; ++v) {
            row_cols(v, buf);
            std::copy(buf.begin(), buf.end(), hp.col_idx.begin() + hp.row_ptr[v]);
        }
    });
    auto slot_of = [&](int32_t r, int32_t c) -> uint32_t {
        const int32_t *b = hp.col_idx.data() + hp.row_ptr[r];
        const int32_t *e = hp.col_idx.data() + hp.row_ptr[r + 1];
        return uint32_t(std::lower_bound(b, e, c) - hp.col_idx.data());
    };
    // 3. permutation (upper-triangle slot of every distinct symmetric pair)
    std::vector<int> pa, pb;
    for (int a = 0; a < np; ++a)
        for (int b = a; b < np; ++b) {
            pa.push_back(a);
            pb.push_back(b);
        }
    hp.perm_sym.resize(size_t(ns) * n_elem);
    parallel_for(n_elem, [&](int64_t lo, int64_t hi) {
        for (int64_t e = lo; e < hi; ++e)
            for (int s = 0; s < ns; ++s) {
                const int32_t i = conn[size_t(pa[s]) * n_elem + e], j = conn[size_t(pb[s]) * n_elem + e];
                hp.perm_sym[size_t(s) * n_elem + e] = slot_of(std::min(i, j), std::max(i, j));
            }
    });
    // mirror slot of every slot (the pattern is structurally symmetric)
    hp.mirror.resize(hp.nnz);
    parallel_for(n_nodes, [&](int64_t lo, int64_t hi) {
        for (int64_t r = lo; r < hi; ++r)
            for (int64_t t = hp.row_ptr[r]; t < hp.row_ptr[r + 1]; ++t) hp.mirror[t] = slot_of(hp.col_idx[t], int32_t(r));
    });
    return QXA_OK;
}

}  // namespace qxa

// Tile plan for the fused formation + scatter kernel (Algorithm 2 after its
// reference tables, in one pass over the mesh).
//
// Elements are ordered along a Morton curve of their centroids and cut into
// tiles of T consecutive elements. One workgroup forms the element matrices
// of a tile in LDS and reduces, for every CSR slot the tile touches, the
// tile's contributions in a fixed order. A slot whose contributions all come
// from one tile is written by that tile (upper slot and its mirror); a slot
// touched by several tiles gets one partial per tile, and the fix-up kernel
// sums the partials in ascending tile order. Every slot is written exactly
// once, with no atomics, so results are bitwise reproducible.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <thread>

#include "qxa_internal.hpp"

namespace qxa {

template <class F>
static void parallel_for(int64_t n, F &&f)
{
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 64 || nt == 1) {
        f(int64_t(0), n);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        int64_t lo = std::min<int64_t>(n, t * chunk), hi = std::min<int64_t>(n, lo + chunk);
        if (lo < hi) th.emplace_back([&f, lo, hi] { f(lo, hi); });
    }
    for (auto &x : th) x.join();
}

static uint64_t spread_bits(uint64_t x, int dim)
{
    // interleave: bit b of x goes to bit dim*b
    uint64_t r = 0;
    for (int b = 0; b < 21; ++b) r |= ((x >> b) & 1ull) << (dim * b);
    return r;
}

qxa_status build_tile_plan(int dim, int order, int64_t n_nodes, int64_t n_elem, const int32_t *conn,
                           const double *coords, const HostPlan &hp, int T, bool pair_units, TilePlan &tp)
{
    const int np = n_local(dim, order), ns = n_sym(np);
    if (int64_t(T + 1) * ns >= 0xffff) return fail(QXA_E_UNSUPPORTED, "tile too large for 16-bit LDS indices");
    tp.T = T;
    tp.n_tiles = (n_elem + T - 1) / T;
    // 1. Morton order of element centroids (vertices only: the map is affine)
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int k = 0; k < dim; ++k)
        for (int64_t v = 0; v < n_nodes; ++v) {
            lo[k] = std::min(lo[k], coords[size_t(k) * n_nodes + v]);
            hi[k] = std::max(hi[k], coords[size_t(k) * n_nodes + v]);
        }
    const int bits = dim == 2 ? 21 : 21;
    const double scale = double((1u << bits) - 1);
    std::vector<std::pair<uint64_t, int32_t>> key(n_elem);
    parallel_for(n_elem, [&](int64_t a, int64_t b) {
        for (int64_t e = a; e < b; ++e) {
            uint64_t code = 0;
            for (int k = 0; k < dim; ++k) {
                double c = 0.0;
                for (int i = 0; i <= dim; ++i) c += coords[size_t(k) * n_nodes + conn[size_t(i) * n_elem + e]];
                c /= (dim + 1);
                const double t = (hi[k] > lo[k]) ? (c - lo[k]) / (hi[k] - lo[k]) : 0.0;
                const uint64_t q = uint64_t(std::min(scale, std::max(0.0, std::floor(t * scale))));
                code |= spread_bits(q, dim) << k;
            }
            key[e] = {code, int32_t(e)};
        }
    });
    std::sort(key.begin(), key.end());
    tp.elem_order.resize(n_elem);
    for (int64_t p = 0; p < n_elem; ++p) tp.elem_order[p] = key[p].second;
    key.clear();
    key.shrink_to_fit();
    tp.tconn.resize(size_t(np) * n_elem);
    parallel_for(n_elem, [&](int64_t a, int64_t b) {
        for (int64_t p = a; p < b; ++p)
            for (int i = 0; i < np; ++i)
                tp.tconn[size_t(i) * n_elem + p] = conn[size_t(i) * n_elem + tp.elem_order[p]];
    });
    // 2. per tile: sorted (upper slot, local element, pair) triples
    const int64_t nt = tp.n_tiles;
    auto tile_entries = [&](int64_t t, std::vector<uint64_t> &buf) {
        // key = slot (32 bits) | lds index (16 bits): lds index = s*T + local element
        buf.clear();
        const int64_t p0 = t * T, p1 = std::min<int64_t>(n_elem, p0 + T);
        for (int64_t p = p0; p < p1; ++p) {
            const int64_t e = tp.elem_order[p];
            for (int s = 0; s < ns; ++s) {
                const uint64_t slot = hp.perm_sym[size_t(s) * n_elem + e];
                const uint64_t lds = uint64_t(s) * (T + 1) + uint64_t(p - p0);
                // order within a slot: ascending local element, then pair
                const uint64_t ord = uint64_t(p - p0) * ns + s;
                buf.push_back((slot << 32) | (ord << 16) | lds);
            }
        }
        std::sort(buf.begin(), buf.end());
    };
    // Records hold at most 6 contributions. A slot is owned by a tile when
    // that tile alone touches it with at most 6 contributions; otherwise
    // (several tiles, or more than 6 contributions in one tile) every tile
    // touching it writes ceil(k / 6) partials of its k contributions, and the
    // fix-up sums them.
    auto chunks = [](size_t k) { return uint32_t((k + 5) / 6); };
    std::vector<std::atomic<uint32_t>> touch(hp.nnz), npart(hp.nnz);
    std::vector<std::atomic<uint8_t>> big(hp.nnz);
    for (int64_t u = 0; u < hp.nnz; ++u) {
        touch[u].store(0, std::memory_order_relaxed);
        npart[u].store(0, std::memory_order_relaxed);
        big[u].store(0, std::memory_order_relaxed);
    }
    parallel_for(nt, [&](int64_t a, int64_t b) {
        std::vector<uint64_t> buf;
        for (int64_t t = a; t < b; ++t) {
            tile_entries(t, buf);
            size_t k = 0;
            while (k < buf.size()) {
                const uint32_t u = uint32_t(buf[k] >> 32);
                size_t k1 = k;
                while (k1 < buf.size() && uint32_t(buf[k1] >> 32) == u) ++k1;
                touch[u].fetch_add(1, std::memory_order_relaxed);
                npart[u].fetch_add(chunks(k1 - k), std::memory_order_relaxed);
                if (k1 - k > 6) big[u].store(1, std::memory_order_relaxed);
                k = k1;
            }
        }
    });
    // shared slots in CSR order; partials numbered by (slot, tile, chunk)
    std::vector<int32_t> sh_id(hp.nnz, -1);
    std::vector<uint32_t> sh_slot;
    tp.part_ptr.assign(1, 0);
    for (int64_t u = 0; u < hp.nnz; ++u)
        if (touch[u].load() > 1 || big[u].load()) {
            sh_id[u] = int32_t(sh_slot.size());
            sh_slot.push_back(uint32_t(u));
            tp.part_ptr.push_back(tp.part_ptr.back() + int64_t(npart[u].load()));
        }
    tp.n_shared = int64_t(sh_slot.size());
    tp.n_partials = tp.part_ptr.back();
    if (tp.n_partials >= (int64_t(1) << 31)) return fail(QXA_E_UNSUPPORTED, "too many partials");
    // output units per tile: owned outputs (upper and mirror) sorted by CSR slot,
    // then the tile's partials; a partial's index is fixed in a second,
    // sequential pass over the tiles in ascending order
    std::vector<std::vector<uint32_t>> trec(nt);
    std::vector<int64_t> tshort(nt, 0);  // pair units at the start of each tile
    std::vector<std::vector<std::pair<uint32_t, uint32_t>>> tpart(nt);  // (shared id, word of its target)
    struct Out {
        uint32_t tgt;  // CSR slot (owned) or shared id
        bool shared;
        int n;  // contributions
        std::array<uint16_t, 6> c;
    };
    parallel_for(nt, [&](int64_t a, int64_t b) {
        std::vector<uint64_t> buf;
        std::vector<Out> owned, shared, S, L;
        for (int64_t t = a; t < b; ++t) {
            tile_entries(t, buf);
            owned.clear();
            shared.clear();
            size_t k = 0;
            while (k < buf.size()) {
                const uint32_t u = uint32_t(buf[k] >> 32);
                size_t k1 = k;
                while (k1 < buf.size() && uint32_t(buf[k1] >> 32) == u) ++k1;
                for (size_t c0 = k; c0 < k1; c0 += 6) {
                    Out o{0u, false, int(std::min(k1, c0 + 6) - c0), {}};
                    o.c.fill(uint16_t(T));  // absent: the zero kept at (pair 0, column T)
                    for (int q = 0; q < o.n; ++q) o.c[q] = uint16_t(buf[c0 + q] & 0xffff);
                    if (sh_id[u] < 0) {
                        o.tgt = u;
                        owned.push_back(o);
                        if (hp.mirror[u] != u) {
                            o.tgt = hp.mirror[u];
                            owned.push_back(o);
                        }
                    } else {
                        o.tgt = uint32_t(sh_id[u]);
                        o.shared = true;
                        shared.push_back(o);
                    }
                }
                k = k1;
            }
            std::sort(owned.begin(), owned.end(), [](const Out &x, const Out &y) { return x.tgt < y.tgt; });
            // outputs with at most two contributions go two to a unit, the rest one
            // to a unit; owned outputs before partials in each group
            S.clear();
            L.clear();
            for (const auto *grp : {&owned, &shared})
                for (const Out &o : *grp) (pair_units && o.n <= 2 ? S : L).push_back(o);
            if (S.size() % 2) {
                L.insert(L.begin(), S.back());
                S.pop_back();
            }
            auto &R = trec[t];
            R.clear();
            tpart[t].clear();
            const size_t us = S.size() / 2;
            tshort[t] = int64_t(us);
            auto target = [&](const Out &o) {
                if (o.shared) tpart[t].push_back({o.tgt, uint32_t(R.size())});
                return o.shared ? 0u : o.tgt;
            };
            auto pack = [](const Out &o, int q) { return uint32_t(o.c[q]) | (uint32_t(o.c[q + 1]) << 16); };
            // unit l: outputs l and l + us, so that each store of a round covers consecutive outputs
            for (size_t l = 0; l < us; ++l) {
                R.push_back(target(S[l]));
                R.push_back(pack(S[l], 0));
                R.push_back(target(S[l + us]));
                R.push_back(pack(S[l + us], 0));
            }
            for (const Out &o : L) {
                R.push_back(target(o));
                R.push_back(pack(o, 0));
                R.push_back(pack(o, 2));
                R.push_back(pack(o, 4));
            }
        }
    });
    {
        std::vector<int64_t> fill(tp.part_ptr.begin(), tp.part_ptr.end() - 1);
        for (int64_t t = 0; t < nt; ++t)
            for (auto &pr : tpart[t]) trec[t][pr.second] = uint32_t(-(fill[pr.first]++) - 1);
    }
    tp.rec_ptr.assign(nt + 1, 0);
    tp.rec_mid.assign(nt, 0);
    for (int64_t t = 0; t < nt; ++t) {
        tp.rec_ptr[t + 1] = tp.rec_ptr[t] + int64_t(trec[t].size() / 4);
        tp.rec_mid[t] = tp.rec_ptr[t] + tshort[t];
    }
    tp.rec.resize(4 * size_t(tp.rec_ptr[nt]));
    parallel_for(nt, [&](int64_t a, int64_t b) {
        for (int64_t t = a; t < b; ++t) std::copy(trec[t].begin(), trec[t].end(), tp.rec.begin() + 4 * tp.rec_ptr[t]);
    });
    // fix-up: every shared upper slot (CSR order) and its mirror
    tp.fix_target.resize(sh_slot.size());
    tp.fix_mirror.resize(sh_slot.size());
    for (size_t k = 0; k < sh_slot.size(); ++k) {
        tp.fix_target[k] = int32_t(sh_slot[k]);
        tp.fix_mirror[k] = int32_t(hp.mirror[sh_slot[k]]);
    }
    return QXA_OK;
}

}  // namespace qxa

namespace qxa {

// Structural check of a tile plan against the pattern: every index the fused
// and fix-up kernels use is in bounds, every CSR slot is written exactly once
// (by one tile or by the fix-up), every partial is written by exactly one tile
// and summed by exactly one shared slot, and every element entry is reduced
// exactly once. Runs on the host before the plan is used.
qxa_status check_tile_plan(int np, int64_t n_elem, const HostPlan &hp, const TilePlan &tp)
{
    const int ns = n_sym(np);
    const int64_t T = tp.T, TP = T + 1;
    std::vector<uint8_t> slot_w(hp.nnz, 0), part_w(tp.n_partials, 0), used;
    if (int64_t(tp.rec_ptr.size()) != tp.n_tiles + 1 || tp.rec_ptr[0] != 0 ||
        int64_t(tp.rec_mid.size()) != tp.n_tiles ||
        int64_t(tp.rec.size()) != 4 * tp.rec_ptr[tp.n_tiles] || int64_t(tp.part_ptr.size()) != tp.n_shared + 1 ||
        tp.part_ptr[0] != 0 || tp.part_ptr[tp.n_shared] != tp.n_partials)
        return fail(QXA_E_INVALID, "tile plan: bad sizes");
    auto write_slot = [&](int64_t g) -> bool { return g >= 0 && g < hp.nnz && slot_w[g]++ == 0; };
    for (int64_t t = 0; t < tp.n_tiles; ++t) {
        const int64_t p0 = t * T, nloc = std::min<int64_t>(T, n_elem - p0);
        used.assign(size_t(TP) * ns, 0);
        if (tp.rec_mid[t] < tp.rec_ptr[t] || tp.rec_mid[t] > tp.rec_ptr[t + 1])
            return fail(QXA_E_INVALID, "tile plan: bad pair-unit range");
        // one output: target g and nc contribution indices
        auto check_out = [&](int32_t g, const uint32_t *c, int nc) -> qxa_status {
            int n = 0;
            for (int q = 0; q < nc; ++q) {
                if (c[q] == uint32_t(T)) continue;  // absent
                if (c[q] >= uint32_t(TP * ns) || int64_t(c[q] % TP) >= nloc)
                    return fail(QXA_E_INVALID, "tile plan: LDS index out of range");
                used[c[q]] = 1;
                ++n;
            }
            if (n == 0) return fail(QXA_E_INVALID, "tile plan: empty record");
            if (g >= 0) {
                if (!write_slot(g)) return fail(QXA_E_INVALID, "tile plan: slot written twice");
            } else {
                const int64_t pi = -int64_t(g) - 1;
                if (pi >= tp.n_partials || part_w[pi]++) return fail(QXA_E_INVALID, "tile plan: partial written twice");
            }
            return QXA_OK;
        };
        for (int64_t r = tp.rec_ptr[t]; r < tp.rec_ptr[t + 1]; ++r) {
            const uint32_t *R = &tp.rec[4 * r];
            qxa_status st;
            if (r < tp.rec_mid[t]) {  // two outputs of at most two contributions
                const uint32_t a[2] = {R[1] & 0xffffu, R[1] >> 16}, b[2] = {R[3] & 0xffffu, R[3] >> 16};
                st = check_out(int32_t(R[0]), a, 2);
                if (!st) st = check_out(int32_t(R[2]), b, 2);
            } else {
                const uint32_t c[6] = {R[1] & 0xffffu, R[1] >> 16, R[2] & 0xffffu, R[2] >> 16, R[3] & 0xffffu, R[3] >> 16};
                st = check_out(int32_t(R[0]), c, 6);
            }
            if (st) return st;
        }
        for (int64_t k = 0; k < nloc; ++k)
            for (int s = 0; s < ns; ++s)
                if (!used[size_t(s) * TP + k]) return fail(QXA_E_INVALID, "tile plan: contribution never reduced");
    }
    for (int64_t k = 0; k < tp.n_shared; ++k)
        if (tp.part_ptr[k + 1] - tp.part_ptr[k] < 2) return fail(QXA_E_INVALID, "tile plan: shared slot with < 2 partials");
    if (int64_t(tp.fix_target.size()) != tp.n_shared || int64_t(tp.fix_mirror.size()) != tp.n_shared)
        return fail(QXA_E_INVALID, "tile plan: bad fix-up sizes");
    for (int64_t k = 0; k < tp.n_shared; ++k) {
        const int32_t u = tp.fix_target[k], m = tp.fix_mirror[k];
        if (k > 0 && u <= tp.fix_target[k - 1]) return fail(QXA_E_INVALID, "tile plan: fix-up not sorted");
        if (u < 0 || u >= hp.nnz || m < 0 || m >= hp.nnz || hp.mirror[u] != uint32_t(m))
            return fail(QXA_E_INVALID, "tile plan: bad fix-up slot");
        if (!write_slot(u)) return fail(QXA_E_INVALID, "tile plan: fix-up slot written twice");
        if (m != u && !write_slot(m)) return fail(QXA_E_INVALID, "tile plan: fix-up mirror written twice");
    }
    for (int64_t k = 0; k < tp.n_partials; ++k)
        if (part_w[k] != 1) return fail(QXA_E_INVALID, "tile plan: partial not written exactly once");
    for (int64_t t = 0; t < hp.nnz; ++t)
        if (slot_w[t] != 1) return fail(QXA_E_INVALID, "tile plan: CSR slot not written exactly once");
    return QXA_OK;
}

}  // namespace qxa

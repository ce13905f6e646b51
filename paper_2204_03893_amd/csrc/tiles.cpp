// Tile plan of the fused formation + scatter kernel (Algorithm 2 after its
// reference tables, in one pass over the mesh).
//
// Elements are ordered along a Morton curve of their centroids and cut into
// tiles of T consecutive elements; consecutive tiles form chains, one chain
// per workgroup of a launch. A workgroup forms the element matrices of its
// tiles one after the other in LDS and reduces, for every CSR slot a tile
// touches, the tile's contributions in a fixed order:
//  - a slot touched by one tile only is written by that tile (upper slot and
//    its mirror);
//  - a slot touched by several tiles of one chain is carried: the first of
//    those tiles writes its partial sum to an LDS carry entry, each later one
//    adds the carry to its own contributions, and the last one writes the
//    CSR value (or, for a slot that other chains touch too, a partial);
//  - a slot touched by several chains gets one partial per chain (or per
//    tile, when no carry entry is free), and the fix-up kernel sums the
//    partials of each such slot in ascending tile order.
// Every slot is written exactly once and nothing is atomic, so results are
// bitwise reproducible.
//
// A tile's outputs travel in 16-byte units (plan_format.hpp).
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <numeric>
#include <queue>
#include <thread>

#include "qxa_internal.hpp"

namespace qxa {


static uint64_t spread_bits(uint64_t x, int dim)
{
    // interleave: bit b of x goes to bit dim*b
    uint64_t r = 0;
    for (int b = 0; b < 21; ++b) r |= ((x >> b) & 1ull) << (dim * b);
    return r;
}

namespace {

// Role of one tile for one upper slot it touches.
enum Role : uint8_t {
    R_OWNED,      // only toucher: CSR upper + mirror
    R_CARRY_OUT,  // first tile of a carried group: carry := own
    R_CARRY_MID,  // carry := carry + own
    R_CARRY_CSR,  // last tile, the slot's only group: CSR := carry + own (upper + mirror)
    R_CARRY_PART, // last tile of a group of a shared slot: partial := carry + own
    R_PART,       // partial := own (uncarried group, or a single tile of a shared slot)
};

struct Group {
    int32_t chain, t_first, t_last, carry;  // carry index or -1
};

}  // namespace

// Stable LSD radix sort of packed (slot << 32 | low) keys by the slot, in digits
// of 11 bits over the range of slots present.
static void radix_sort_by_slot(uint64_t *a, uint64_t *a_end, std::vector<uint64_t> &tmp)
{
    const size_t n = size_t(a_end - a);
    if (n < 2) return;
    uint32_t lo = UINT32_MAX, hi = 0;
    for (size_t k = 0; k < n; ++k) {
        const uint32_t u = uint32_t(a[k] >> 32);
        lo = std::min(lo, u);
        hi = std::max(hi, u);
    }
    const uint32_t range = hi - lo;
    const int bits = range ? 32 - __builtin_clz(range) : 0;
    tmp.resize(n);
    uint64_t *src = a, *dst = tmp.data();
    for (int shift = 0; shift < bits; shift += 11) {
        uint32_t cnt[2049] = {};
        for (size_t k = 0; k < n; ++k) ++cnt[((uint32_t(src[k] >> 32) - lo) >> shift & 2047u) + 1];
        for (int d = 0; d < 2048; ++d) cnt[d + 1] += cnt[d];
        for (size_t k = 0; k < n; ++k) dst[cnt[(uint32_t(src[k] >> 32) - lo) >> shift & 2047u]++] = src[k];
        std::swap(src, dst);
    }
    if (src != a) std::copy(src, src + n, a);
}

qxa_status build_tile_plan(int dim, int order, int64_t n_nodes, int64_t n_elem, const int32_t *conn,
                           const double *coords, const HostPlan &hp, const TileParams &prm, TilePlan &tp)
{
    const int np = n_local(dim, order), ns = n_sym(np);
    const int T = prm.T;
    if (int64_t(T) * ns >= 0xffff) return fail(QXA_E_UNSUPPORTED, "tile too large for 16-bit LDS indices");
    tp = TilePlan{};
    tp.T = T;
    tp.n_tiles = (n_elem + T - 1) / T;
    tp.carry_cap = std::max(0, std::min(prm.carry_cap, 0xffff - carry_base(ns, T)));
    const int64_t nt = tp.n_tiles;
    // 1. Morton order of element centroids (vertices only: the map is affine)
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int k = 0; k < dim; ++k)
        for (int64_t v = 0; v < n_nodes; ++v) {
            lo[k] = std::min(lo[k], coords[size_t(k) * n_nodes + v]);
            hi[k] = std::max(hi[k], coords[size_t(k) * n_nodes + v]);
        }
    const double scale = double((1u << 21) - 1);
    hvec<std::pair<uint64_t, int32_t>> key(n_elem);
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
    parallel_sort(key.begin(), key.end());  // (code, element): no ties
    tp.elem_order.resize(n_elem);
    parallel_for(n_elem, [&](int64_t a, int64_t b) {
        for (int64_t p = a; p < b; ++p) tp.elem_order[p] = key[p].second;
    });
    key.clear();
    key.shrink_to_fit();
    // Runs (carry entries too few for long chains: 3D P2, 3D P3). The full tiles are
    // renumbered so that chain c = (XCD x, workgroup i) = (c / W, c % W), W = chains / 8,
    // holds from every row of W L consecutive Morton tiles of XCD x's eighth the run of L
    // tiles i L .. i L + L - 1. The workgroups of one XCD then work on one row at a time
    // (neighbouring tiles at the same time, as in the side-by-side walk, so that their
    // writes to shared CSR lines meet in that XCD's L2), and each passes the slots its
    // run's tiles share through carry entries. A partial last tile stays last (in the
    // last chain). Too few tiles for a run per workgroup: one-tile chains.
    const int64_t nfull = n_elem / T;
    const bool runs = prm.run_len > 1 && prm.chains >= 8 && prm.chains % 8 == 0 &&
                      nfull >= prm.chains * int64_t(prm.run_len) && nt > 0;
    std::vector<int64_t> run_chain_len;
    if (runs) {
        const int64_t W = prm.chains / 8, L = prm.run_len;
        std::vector<int64_t> order;  // new tile -> Morton tile
        order.reserve(size_t(nfull));
        run_chain_len.assign(size_t(prm.chains), 0);
        for (int64_t x = 0; x < 8; ++x) {
            const int64_t x0 = x * nfull / 8, n = (x + 1) * nfull / 8 - x0;
            for (int64_t i = 0; i < W; ++i)
                for (int64_t r = 0; r * W * L < n; ++r)
                    for (int64_t l = 0; l < L; ++l) {
                        const int64_t m = r * W * L + i * L + l;
                        if (m >= n) break;
                        order.push_back(x0 + m);
                        ++run_chain_len[size_t(x * W + i)];
                    }
        }
        if (nt > nfull) ++run_chain_len.back();  // the partial tile
        hvec<int32_t> eo(n_elem);
        parallel_for(nfull, [&](int64_t a, int64_t b) {
            for (int64_t t = a; t < b; ++t)
                std::copy(tp.elem_order.begin() + order[t] * T, tp.elem_order.begin() + (order[t] + 1) * T,
                          eo.begin() + t * T);
        });
        std::copy(tp.elem_order.begin() + nfull * T, tp.elem_order.end(), eo.begin() + nfull * T);
        tp.elem_order.swap(eo);
    }
    tp.tconn.resize(size_t(np) * n_elem);
    parallel_for(n_elem, [&](int64_t a, int64_t b) {
        for (int64_t p = a; p < b; ++p)
            for (int i = 0; i < np; ++i)
                tp.tconn[size_t(i) * n_elem + p] = conn[size_t(i) * n_elem + tp.elem_order[p]];
    });
    // 2. chains: nc balanced runs of consecutive tiles (or the runs above; with run_len > 1
    //    and too few tiles for them, one-tile chains)
    const int64_t nc = nt == 0 ? 0
                       : runs ? prm.chains
                       : prm.run_len > 1 ? nt
                              : std::max<int64_t>(1, std::min<int64_t>(nt, prm.chains));
    tp.chain_ptr.assign(nc + 1, 0);
    for (int64_t c = 1; c <= nc; ++c)
        tp.chain_ptr[c] = runs ? tp.chain_ptr[c - 1] + run_chain_len[size_t(c - 1)] : c * nt / nc;
    std::vector<int32_t> chain_of(nt);
    for (int64_t c = 0; c < nc; ++c)
        for (int64_t t = tp.chain_ptr[c]; t < tp.chain_ptr[c + 1]; ++t) chain_of[t] = int32_t(c);
    // 3. per tile: sorted (upper slot, plan order, LDS index) triples, kept for
    //    the passes below at ent[p0 * ns ..] (p0 the tile's first position); the
    //    plan order within a slot is ascending local element, then pair
    hvec<uint64_t> ent(size_t(n_elem) * ns);
    parallel_for(nt, [&](int64_t a, int64_t b) {
        std::vector<uint64_t> tmp;
        for (int64_t t = a; t < b; ++t) {
            const int64_t p0 = t * T, p1 = std::min<int64_t>(n_elem, p0 + T);
            uint64_t *out = ent.data() + size_t(p0) * ns;
            for (int64_t p = p0; p < p1; ++p) {
                const int64_t e = tp.elem_order[p];
                for (int s = 0; s < ns; ++s) {
                    const uint64_t slot = hp.perm_sym[size_t(s) * n_elem + e];
                    const uint64_t lds = uint64_t(s) * (T + 1) + uint64_t(p - p0);
                    const uint64_t ord = uint64_t(p - p0) * ns + s;
                    *out++ = (slot << 32) | (ord << 16) | lds;
                }
            }
            // entries are written in plan order (ascending ord), so a stable sort by slot
            // alone gives the (slot, ord) order
            radix_sort_by_slot(ent.data() + size_t(p0) * ns, out, tmp);
        }
    }, 16);
    auto tile_span = [&](int64_t t, const uint64_t *&b, const uint64_t *&e) {
        b = ent.data() + size_t(t) * T * ns;
        e = ent.data() + size_t(std::min<int64_t>(n_elem, (t + 1) * T)) * ns;
    };
    // the distinct slots of a tile: f(slot, first entry, end of its entries)
    auto for_slots = [&](int64_t t, auto &&f) {
        const uint64_t *b, *e;
        tile_span(t, b, e);
        for (const uint64_t *k = b; k < e;) {
            const uint32_t u = uint32_t(*k >> 32);
            const uint64_t *k1 = k + 1;
            while (k1 < e && uint32_t(*k1 >> 32) == u) ++k1;
            f(u, k, k1);
            k = k1;
        }
    };
    // 4. tiles touching every upper slot; afterwards the same array holds the
    //    slot's index among the multi-tile slots (-1: one tile)
    const int64_t nnz = hp.nnz;
    hvec<int32_t> mid(nnz);
    parallel_for(nnz, [&](int64_t a, int64_t b) { std::fill(mid.begin() + a, mid.begin() + b, 0); });
    parallel_for(nt, [&](int64_t a, int64_t b) {
        for (int64_t t = a; t < b; ++t)
            for_slots(t, [&](uint32_t u, const uint64_t *, const uint64_t *) {
                __atomic_fetch_add(&mid[u], 1, __ATOMIC_RELAXED);
            });
    }, 16);
    // 5. multi-tile slots (ascending slot order): their touching tiles, sorted,
    //    and their chain groups
    const unsigned nth = host_threads();
    const int64_t uchunk = (nnz + nth - 1) / nth;
    std::vector<int64_t> cbase(nth + 1, 0);
    parallel_for(nth, [&](int64_t a, int64_t b) {
        for (int64_t c = a; c < b; ++c) {
            int64_t n = 0;
            for (int64_t u = c * uchunk; u < std::min(nnz, (c + 1) * uchunk); ++u) n += mid[u] > 1;
            cbase[c + 1] = n;
        }
    }, 0);
    for (unsigned c = 0; c < nth; ++c) cbase[c + 1] += cbase[c];
    const int64_t nm = cbase[nth];
    hvec<uint32_t> mslot(nm);
    hvec<int64_t> mptr(nm + 1);
    mptr[0] = 0;
    parallel_for(nth, [&](int64_t a, int64_t b) {
        for (int64_t c = a; c < b; ++c) {
            int64_t m = cbase[c];
            for (int64_t u = c * uchunk; u < std::min(nnz, (c + 1) * uchunk); ++u) {
                if (mid[u] > 1) {
                    mslot[m] = uint32_t(u);
                    mptr[m + 1] = mid[u];
                    mid[u] = int32_t(m++);
                } else {
                    mid[u] = -1;
                }
            }
        }
    }, 0);
    for (int64_t m = 0; m < nm; ++m) mptr[m + 1] += mptr[m];
    hvec<int32_t> mtiles(mptr[nm]);
    {
        hvec<int32_t> cur(nm);
        parallel_for(nm, [&](int64_t a, int64_t b) { std::fill(cur.begin() + a, cur.begin() + b, 0); });
        parallel_for(nt, [&](int64_t a, int64_t b) {
            for (int64_t t = a; t < b; ++t)
                for_slots(t, [&](uint32_t u, const uint64_t *, const uint64_t *) {
                    const int32_t m = mid[u];
                    if (m >= 0) mtiles[mptr[m] + __atomic_fetch_add(&cur[m], 1, __ATOMIC_RELAXED)] = int32_t(t);
                });
        }, 16);
    }
    // without carries (no entries, or chains of one tile) every multi-tile slot is a
    // partial per tile and no chain groups are needed
    const bool carries = tp.carry_cap > 0 && nc < nt;
    hvec<int64_t> gptr(carries ? nm + 1 : 1);
    gptr[0] = 0;
    hvec<Group> groups;
    parallel_for(nm, [&](int64_t a, int64_t b) {
        for (int64_t m = a; m < b; ++m) std::sort(mtiles.begin() + mptr[m], mtiles.begin() + mptr[m + 1]);
    });
    if (carries) {
        hvec<int32_t> ngr(nm);
        parallel_for(nm, [&](int64_t a, int64_t b) {
            for (int64_t m = a; m < b; ++m) {
                int g = 1;
                for (int64_t k = mptr[m] + 1; k < mptr[m + 1]; ++k) g += chain_of[mtiles[k]] != chain_of[mtiles[k - 1]];
                ngr[m] = g;
            }
        });
        for (int64_t m = 0; m < nm; ++m) gptr[m + 1] = gptr[m] + ngr[m];
        groups.resize(gptr[nm]);
        parallel_for(nm, [&](int64_t a, int64_t b) {
            for (int64_t m = a; m < b; ++m) {
                int64_t g = gptr[m];
                for (int64_t k = mptr[m]; k < mptr[m + 1]; ++k) {
                    const int32_t t = mtiles[k], c = chain_of[t];
                    if (k == mptr[m] || c != chain_of[mtiles[k - 1]]) groups[g++] = Group{c, t, t, -1};
                    else groups[g - 1].t_last = t;
                }
            }
        });
    }
    // 6. carry entries, per chain in tile order: a group spanning tiles
    //    t_first < t_last holds an entry from t_first to t_last; an entry read
    //    (for the last time) in tile t is free again from tile t + 1. A group
    //    that finds no free entry is not carried (one partial per tile).
    std::vector<std::vector<int64_t>> chain_groups(carries ? nc : 0);  // group indices spanning > 1 tile
    for (int64_t g = 0; g < int64_t(groups.size()); ++g)
        if (groups[g].t_first < groups[g].t_last) chain_groups[groups[g].chain].push_back(g);
    std::vector<int32_t> chain_used(carries ? nc : 0, 0);
    parallel_for(int64_t(chain_groups.size()), [&](int64_t a, int64_t b) {
        for (int64_t c = a; c < b; ++c) {
            auto &L = chain_groups[c];
            std::sort(L.begin(), L.end(), [&](int64_t x, int64_t y) {
                return groups[x].t_first != groups[y].t_first ? groups[x].t_first < groups[y].t_first : x < y;
            });
            std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> freeq;
            for (int32_t k = 0; k < tp.carry_cap; ++k) freeq.push(k);
            // live entries ordered by their last tile
            std::priority_queue<std::pair<int32_t, int32_t>, std::vector<std::pair<int32_t, int32_t>>,
                                std::greater<std::pair<int32_t, int32_t>>>
                live;
            int32_t used = 0;
            for (int64_t g : L) {
                Group &G = groups[g];
                while (!live.empty() && live.top().first < G.t_first) {
                    freeq.push(live.top().second);
                    live.pop();
                }
                if (freeq.empty()) continue;
                G.carry = freeq.top();
                freeq.pop();
                live.push({G.t_last, G.carry});
                used = std::max<int32_t>(used, int32_t(live.size()));
            }
            chain_used[c] = used;
        }
    }, 2);
    for (int32_t u : chain_used) tp.carry_used = std::max(tp.carry_used, u);
    // 7. shared slots (a partial at least) and the index of every partial:
    //    one per (tile, slot) of role R_PART or R_CARRY_PART, numbered by slot,
    //    then ascending tile (pidx is parallel to mtiles; -1: no partial)
    auto role_of = [&](uint32_t u, int32_t t, int32_t &carry) -> Role {
        carry = -1;
        const int32_t m = mid[u];
        if (m < 0) return R_OWNED;
        if (!carries) return R_PART;
        const int32_t c = chain_of[t];
        int64_t g = gptr[m];
        while (groups[g].chain != c) ++g;
        const Group &G = groups[g];
        const bool single = gptr[m + 1] - gptr[m] == 1;
        if (G.carry < 0) return R_PART;
        carry = G.carry;
        if (t == G.t_first) return R_CARRY_OUT;
        if (t < G.t_last) return R_CARRY_MID;
        return single ? R_CARRY_CSR : R_CARRY_PART;
    };
    hvec<int32_t> pidx(mptr[nm]);
    hvec<int64_t> mpart(nm + 1);
    mpart[0] = 0;
    parallel_for(nm, [&](int64_t a, int64_t b) {
        for (int64_t m = a; m < b; ++m) {
            int32_t n = 0, carry;
            for (int64_t k = mptr[m]; k < mptr[m + 1]; ++k) {
                const Role r = role_of(mslot[m], mtiles[k], carry);
                pidx[k] = (r == R_PART || r == R_CARRY_PART) ? n++ : -1;
            }
            mpart[m + 1] = n;
        }
    });
    for (int64_t m = 0; m < nm; ++m) mpart[m + 1] += mpart[m];
    tp.n_partials = mpart[nm];
    if (tp.n_partials >= (int64_t(1) << 30)) return fail(QXA_E_UNSUPPORTED, "too many partials");
    if (nnz >= (int64_t(1) << 30)) return fail(QXA_E_UNSUPPORTED, "more than 2^30 CSR slots");
    parallel_for(nm, [&](int64_t a, int64_t b) {
        for (int64_t m = a; m < b; ++m)
            for (int64_t k = mptr[m]; k < mptr[m + 1]; ++k)
                if (pidx[k] >= 0) pidx[k] += int32_t(mpart[m]);
    });
    tp.part_ptr.assign(1, 0);
    std::vector<uint32_t> sh_slot;
    for (int64_t m = 0; m < nm; ++m)
        if (mpart[m + 1] > mpart[m]) {
            sh_slot.push_back(mslot[m]);
            tp.part_ptr.push_back(mpart[m + 1]);
        }
    tp.n_shared = int64_t(sh_slot.size());
    // index of the partial of (tile t, slot u) (a multi-tile slot)
    auto partial_of = [&](uint32_t u, int32_t t) -> int32_t {
        const int32_t m = mid[u];
        const int32_t *b = mtiles.data() + mptr[m], *e = mtiles.data() + mptr[m + 1];
        return pidx[std::lower_bound(b, e, t) - mtiles.data()];
    };
    // 8. outputs of every tile, packed into units. An output of more than six
    //    entries takes k consecutive single units in one block of kSegLanes
    //    units: all but the last carry the code kCodeExt, and the last one
    //    (which has the output's code) adds their sums to its own.
    const uint32_t cb = uint32_t(carry_base(ns, T));
    struct Out {
        int32_t code;
        uint8_t kind;   // 0 CSR, 1 carry, 2 partial
        uint32_t n;     // entries (a carry entry included)
        uint32_t e0;    // first entry in the tile's entry list
    };
    std::atomic<bool> too_long{false};
    std::vector<std::vector<uint32_t>> trec(nt);
    std::vector<int64_t> tpairs(nt, 0), touts(nt, 0), tcin(nt, 0), text(nt, 0), tnone(nt, 0);
    parallel_for(nt, [&](int64_t a, int64_t b) {
        // outputs by kind: CSR upper slots, CSR mirror slots, carries, partials
        std::vector<Out> outs, up, mi, ca, pa, S, L;
        std::vector<uint16_t> ents;
        std::vector<const Out *> B, O;  // single outputs of several units, of one unit
        for (int64_t t = a; t < b; ++t) {
            up.clear();
            mi.clear();
            ca.clear();
            pa.clear();
            ents.clear();
            int64_t n_cin = 0;
            auto add_to = [&](std::vector<Out> &dst, int32_t code, uint8_t kind, int32_t cin, const uint64_t *own,
                              size_t n_own) {
                dst.push_back(Out{code, kind, uint32_t(n_own + (cin >= 0)), uint32_t(ents.size())});
                if (cin >= 0) ents.push_back(uint16_t(cb + uint32_t(cin)));
                for (size_t m = 0; m < n_own; ++m) ents.push_back(uint16_t(own[m] & 0xffff));
                n_cin += cin >= 0;
            };
            for_slots(t, [&](uint32_t u, const uint64_t *own, const uint64_t *own_end) {
                int32_t carry;
                const Role r = role_of(u, int32_t(t), carry);
                const size_t n_own = size_t(own_end - own);
                const int32_t mir = int32_t(hp.mirror[u]);
                switch (r) {
                case R_OWNED:
                    add_to(up, int32_t(u), 0, -1, own, n_own);
                    if (mir != int32_t(u)) add_to(mi, mir, 0, -1, own, n_own);
                    break;
                case R_CARRY_OUT: add_to(ca, kCodeCarry | carry, 1, -1, own, n_own); break;
                case R_CARRY_MID: add_to(ca, kCodeCarry | carry, 1, carry, own, n_own); break;
                case R_CARRY_CSR:
                    add_to(up, int32_t(u), 0, carry, own, n_own);
                    if (mir != int32_t(u)) add_to(mi, mir, 0, carry, own, n_own);
                    break;
                case R_CARRY_PART:
                case R_PART: {
                    const int32_t p = partial_of(u, int32_t(t));
                    add_to(pa, -p - 1, 2, r == R_CARRY_PART ? carry : -1, own, n_own);
                    break;
                }
                }
            });
            tcin[t] = n_cin;
            // CSR outputs (ascending slot), then carries (ascending code), then partials
            // (ascending partial index: codes descending). The slots come in ascending
            // order, and so do the upper slots and the partials (a slot's partials are
            // numbered in slot order); the mirror slots and the carry codes are sorted,
            // and the mirrors merged into the upper slots. Every code is distinct.
            auto by_code = [](const Out &x, const Out &y) { return x.code < y.code; };
            std::sort(mi.begin(), mi.end(), by_code);
            std::sort(ca.begin(), ca.end(), by_code);
            outs.resize(up.size() + mi.size());
            std::merge(up.begin(), up.end(), mi.begin(), mi.end(), outs.begin(), by_code);
            outs.insert(outs.end(), ca.begin(), ca.end());
            outs.insert(outs.end(), pa.begin(), pa.end());
            S.clear();
            L.clear();
            for (const Out &o : outs) (prm.pair_units && o.n <= kPairEntries ? S : L).push_back(o);
            if (S.size() % 2) {
                L.insert(L.begin(), S.back());
                S.pop_back();
            }
            auto &R = trec[t];
            R.clear();
            R.reserve(4 * (outs.size() + ents.size() / kUnitEntries + kSegLanes));
            const size_t us = S.size() / 2;
            tpairs[t] = int64_t(us);
            touts[t] = int64_t(outs.size());
            auto ent = [&](const Out &o, uint32_t q) { return q < o.n ? uint32_t(ents[o.e0 + q]) : uint32_t(T); };
            auto pack = [&](const Out &o, uint32_t q) { return ent(o, q) | (ent(o, q + 1) << 16); };
            // unit l: outputs l and l + us, so that each store of a round covers consecutive outputs
            for (size_t l = 0; l < us; ++l) {
                R.push_back(uint32_t(S[l].code));
                R.push_back(pack(S[l], 0));
                R.push_back(uint32_t(S[l + us].code));
                R.push_back(pack(S[l + us], 0));
            }
            // singles. An output of k > 1 units takes k consecutive units inside one
            // block of kSegLanes units of the tile (one wave's units of a round);
            // first fit, most units first, the one-unit outputs filling in between,
            // so a hole (a unit that stores nothing) only pads a block when no
            // one-unit output is left.
            auto units_of = [](const Out &o) { return (o.n + kUnitEntries - 1) / kUnitEntries; };
            B.clear();
            O.clear();
            for (const Out &o : L) (units_of(o) > 1 ? B : O).push_back(&o);
            std::stable_sort(B.begin(), B.end(),
                             [&](const Out *x, const Out *y) { return units_of(*x) > units_of(*y); });
            size_t b0 = 0, oi = 0;  // first unplaced multi-unit output; next one-unit output
            auto emit = [&](const Out &o) {
                const uint32_t k = units_of(o);
                if (k > uint32_t(kSegLanes)) too_long = true;  // more entries than a tile can hold
                for (uint32_t m = 0; m < k; ++m) {
                    R.push_back(uint32_t(m + 1 == k ? o.code : kCodeExt));
                    R.push_back(pack(o, m * kUnitEntries));
                    R.push_back(pack(o, m * kUnitEntries + 2));
                    R.push_back(pack(o, m * kUnitEntries + 4));
                }
                text[t] += k - 1;
            };
            while (b0 < B.size() || oi < O.size()) {
                const uint32_t room = kSegLanes - uint32_t((R.size() / 4) % kSegLanes);
                size_t j = b0;
                while (j < B.size() && (!B[j] || units_of(*B[j]) > room)) ++j;
                if (j < B.size()) {
                    emit(*B[j]);
                    B[j] = nullptr;
                    while (b0 < B.size() && !B[b0]) ++b0;
                } else if (oi < O.size()) {
                    emit(*O[oi++]);
                } else {
                    ++tnone[t];
                    R.push_back(uint32_t(kCodeNone));
                    R.push_back(uint32_t(T) | (uint32_t(T) << 16));
                    R.push_back(uint32_t(T) | (uint32_t(T) << 16));
                    R.push_back(uint32_t(T) | (uint32_t(T) << 16));
                }
            }
        }
    }, 16);
    if (too_long) return fail(QXA_E_INVALID, "tile plan: an output of more entries than one wave's units hold");
    tp.rec_ptr.assign(nt + 1, 0);
    tp.rec_mid.assign(nt, 0);
    for (int64_t t = 0; t < nt; ++t) {
        tp.rec_ptr[t + 1] = tp.rec_ptr[t] + int64_t(trec[t].size() / 4);
        tp.rec_mid[t] = tp.rec_ptr[t] + tpairs[t];
        tp.n_outputs += touts[t];
        tp.n_carry_reads += tcin[t];
        tp.n_ext_units += text[t];
        tp.n_empty_units += tnone[t];
    }
    tp.rec.resize(4 * size_t(tp.rec_ptr[nt]));
    parallel_for(nt, [&](int64_t a, int64_t b) {
        for (int64_t t = a; t < b; ++t) {
            std::copy(trec[t].begin(), trec[t].end(), tp.rec.begin() + 4 * tp.rec_ptr[t]);
            std::vector<uint32_t>().swap(trec[t]);
        }
    }, 16);
    // fix-up: every shared upper slot (CSR order) and its mirror
    tp.fix_target.resize(sh_slot.size());
    tp.fix_mirror.resize(sh_slot.size());
    parallel_for(int64_t(sh_slot.size()), [&](int64_t a, int64_t b) {
        for (int64_t k = a; k < b; ++k) {
            tp.fix_target[k] = int32_t(sh_slot[k]);
            tp.fix_mirror[k] = int32_t(hp.mirror[sh_slot[k]]);
        }
    });
    return QXA_OK;
}

// Check of a tile plan against the pattern, by executing it on the host with
// exact integer sums: every element entry gets a pseudo-random 64-bit value;
// the tiles of each chain are reduced in order as the kernels reduce them
// (decoding the units as they do), carries in a per-chain array, partials
// written once and summed by the fix-up; the result must equal the sums of
// the element entries of every slot through the element-entry -> slot map,
// on both triangles. It also checks every index the kernels use, that each
// CSR slot and partial is written exactly once, and that within a tile a
// carry entry written by an output is read by no other output, and is read
// only after an earlier tile of the same chain wrote it.
qxa_status check_tile_plan(int np, int64_t n_elem, const HostPlan &hp, const TilePlan &tp)
{
    const int ns = n_sym(np);
    const int64_t T = tp.T, TP = T + 1, nt = tp.n_tiles, nnz = hp.nnz;
    const uint32_t cb = uint32_t(carry_base(ns, int(T)));
    const int64_t nc = int64_t(tp.chain_ptr.size()) - 1;
    if (nt > 0 && (nc < 1 || tp.chain_ptr[0] != 0 || tp.chain_ptr[nc] != nt))
        return fail(QXA_E_INVALID, "tile plan: bad chains");
    for (int64_t c = 0; c < nc; ++c)
        if (tp.chain_ptr[c + 1] <= tp.chain_ptr[c]) return fail(QXA_E_INVALID, "tile plan: empty chain");
    if (int64_t(tp.rec_ptr.size()) != nt + 1 || tp.rec_ptr[0] != 0 || int64_t(tp.rec_mid.size()) != nt ||
        int64_t(tp.rec.size()) != 4 * tp.rec_ptr[nt] || int64_t(tp.part_ptr.size()) != tp.n_shared + 1 ||
        tp.part_ptr[0] != 0 || tp.part_ptr[tp.n_shared] != tp.n_partials ||
        int64_t(tp.fix_target.size()) != tp.n_shared || int64_t(tp.fix_mirror.size()) != tp.n_shared ||
        tp.carry_used > tp.carry_cap || int64_t(cb) + tp.carry_cap > 0xffff)
        return fail(QXA_E_INVALID, "tile plan: bad sizes");
    auto value = [](uint64_t s, uint64_t e) {
        uint64_t x = (s << 40) ^ (e * 0x9E3779B97F4A7C15ull) ^ 0xD1B54A32D192ED03ull;
        x ^= x >> 31;
        x *= 0xBF58476D1CE4E5B9ull;
        x ^= x >> 29;
        return x;
    };
    // expected sums (wrapping 64-bit adds, so their order does not matter),
    // write counts of every slot and partial
    hvec<uint64_t> expect(nnz), part(tp.n_partials);
    hvec<uint8_t> is_up(nnz), slot_ws(nnz), part_ws(tp.n_partials);
    parallel_for(nnz, [&](int64_t a, int64_t b) {
        std::fill(expect.begin() + a, expect.begin() + b, 0);
        std::fill(is_up.begin() + a, is_up.begin() + b, 0);
        std::fill(slot_ws.begin() + a, slot_ws.begin() + b, 0);
    });
    parallel_for(tp.n_partials, [&](int64_t a, int64_t b) {
        std::fill(part.begin() + a, part.begin() + b, 0);
        std::fill(part_ws.begin() + a, part_ws.begin() + b, 0);
    });
    parallel_for(n_elem, [&](int64_t a, int64_t b) {
        for (int64_t e = a; e < b; ++e)
            for (int s = 0; s < ns; ++s) {
                const uint32_t u = hp.perm_sym[size_t(s) * n_elem + e];
                __atomic_fetch_add(&expect[u], value(s, e), __ATOMIC_RELAXED);
                __atomic_store_n(&is_up[u], uint8_t(1), __ATOMIC_RELAXED);
            }
    });
    auto expected = [&](int64_t u) { return is_up[u] ? expect[u] : expect[hp.mirror[u]]; };
    auto write_once = [](uint8_t &w) { return __atomic_fetch_add(&w, uint8_t(1), __ATOMIC_RELAXED) == 0; };
    std::atomic<int> bad{0};
    std::string why;
    std::mutex why_mu;
    auto flag = [&](const char *msg) {
        std::lock_guard<std::mutex> lk(why_mu);
        if (!bad.exchange(1)) why = msg;
    };
    // chains are independent: their CSR slots, partials and carries are disjoint
    parallel_for(nc, [&](int64_t ca, int64_t cbd) {
        const size_t cap = size_t(std::max(1, tp.carry_cap));
        std::vector<uint64_t> carry(cap, 0);
        std::vector<int64_t> wtile(cap), stamp(cap);    // tile of the last write; tile of the marks below
        std::vector<int64_t> writer(cap), reader(cap);  // this tile's writer / reader output (-2: several readers)
        for (int64_t c = ca; c < cbd && !bad.load(); ++c) {
            std::fill(wtile.begin(), wtile.end(), -1);
            std::fill(stamp.begin(), stamp.end(), -1);
            for (int64_t t = tp.chain_ptr[c]; t < tp.chain_ptr[c + 1] && !bad.load(); ++t) {
                const int64_t p0 = t * T, nloc = std::min<int64_t>(T, n_elem - p0);
                if (tp.rec_mid[t] < tp.rec_ptr[t] || tp.rec_mid[t] > tp.rec_ptr[t + 1]) {
                    flag("tile plan: bad pair-unit range");
                    return;
                }
                auto mark = [&](uint32_t k) {
                    if (stamp[k] != t) {
                        stamp[k] = t;
                        writer[k] = reader[k] = -1;
                    }
                };
                // one unit: code and entries, as a kernel lane reduces it; `pend` is the
                // sum of the output's units before (kCodeExt), oid the output
                auto output = [&](int64_t oid, int32_t code, const uint32_t *c, int n, uint64_t pend,
                                  bool has_pend, uint64_t &acc) -> bool {
                    acc = has_pend ? pend : 0;
                    int used = 0;
                    for (int q = 0; q < n; ++q) {
                        const uint32_t v = c[q];
                        if (v == uint32_t(T)) continue;
                        ++used;
                        if (v >= cb) {
                            const uint32_t k = v - cb;
                            if (q != 0 || has_pend || int(k) >= tp.carry_cap || wtile[k] < 0 || wtile[k] >= t) {
                                flag("tile plan: bad carry read");
                                return false;
                            }
                            mark(k);
                            if (writer[k] >= 0 && writer[k] != oid) {
                                flag("tile plan: carry read and written by different outputs of a tile");
                                return false;
                            }
                            reader[k] = reader[k] == -1 ? oid : -2;
                            acc += carry[k];
                            continue;
                        }
                        if (int64_t(v % TP) >= nloc || v / TP >= uint32_t(ns)) {
                            flag("tile plan: LDS index out of range");
                            return false;
                        }
                        acc += value(v / TP, tp.elem_order[p0 + v % TP]);
                    }
                    if (code == kCodeNone) {
                        if (used || has_pend) {
                            flag("tile plan: a no-op unit with entries");
                            return false;
                        }
                        return true;
                    }
                    if (used == 0 && !has_pend) {
                        flag("tile plan: empty output");
                        return false;
                    }
                    if (code == kCodeExt) return true;
                    if (code >= 0 && code < kCodeCarry) {
                        if (code >= nnz || !write_once(slot_ws[code])) {
                            flag("tile plan: CSR slot written twice or out of range");
                            return false;
                        }
                        if (acc != expected(code)) {
                            flag("tile plan: slot sum differs from the element entries");
                            return false;
                        }
                    } else if (code >= kCodeCarry && code < kCodeCarryEnd) {
                        const uint32_t k = uint32_t(code - kCodeCarry);
                        if (int(k) >= tp.carry_cap) {
                            flag("tile plan: carry index out of range");
                            return false;
                        }
                        mark(k);
                        if (writer[k] != -1 || (reader[k] != -1 && reader[k] != oid)) {
                            flag("tile plan: carry written twice, or read by another output, in a tile");
                            return false;
                        }
                        writer[k] = oid;
                        carry[k] = acc;
                        wtile[k] = t;
                    } else if (code < 0) {
                        const int64_t pi = -int64_t(code) - 1;
                        if (pi >= tp.n_partials || !write_once(part_ws[pi])) {
                            flag("tile plan: partial written twice or out of range");
                            return false;
                        }
                        part[pi] = acc;
                    } else {
                        flag("tile plan: bad target code");
                        return false;
                    }
                    return true;
                };
                // an extended output: the sum of the units before, and their output id
                bool has_pend = false;
                uint64_t pend = 0;
                int64_t pend_oid = 0;
                for (int64_t r = tp.rec_ptr[t]; r < tp.rec_ptr[t + 1]; ++r) {
                    const uint32_t *R = &tp.rec[4 * r];
                    uint64_t acc;
                    if (has_pend && (r - tp.rec_ptr[t]) % kSegLanes == 0) {
                        flag("tile plan: an extended output crosses a block of units");
                        return;
                    }
                    if (r < tp.rec_mid[t]) {
                        const uint32_t a[2] = {R[1] & 0xffffu, R[1] >> 16}, b2[2] = {R[3] & 0xffffu, R[3] >> 16};
                        if (has_pend || int32_t(R[0]) == kCodeExt || int32_t(R[2]) == kCodeExt) {
                            flag("tile plan: a pair unit continues or extends an output");
                            return;
                        }
                        if (!output(2 * r, int32_t(R[0]), a, 2, 0, false, acc) ||
                            !output(2 * r + 1, int32_t(R[2]), b2, 2, 0, false, acc))
                            return;
                    } else {
                        const uint32_t e6[6] = {R[1] & 0xffffu, R[1] >> 16, R[2] & 0xffffu,
                                                R[2] >> 16,     R[3] & 0xffffu, R[3] >> 16};
                        const int64_t oid = has_pend ? pend_oid : 2 * r;
                        if (!output(oid, int32_t(R[0]), e6, 6, pend, has_pend, acc)) return;
                        has_pend = int32_t(R[0]) == kCodeExt;
                        pend = acc;
                        pend_oid = oid;
                    }
                }
                if (has_pend) {
                    flag("tile plan: an extended output without its last unit");
                    return;
                }
            }
        }
    }, 2);

    if (bad.load()) return fail(QXA_E_INVALID, why);
    parallel_for(tp.n_partials, [&](int64_t a, int64_t b) {
        for (int64_t k = a; k < b; ++k)
            if (part_ws[k] != 1) {
                flag("tile plan: partial not written exactly once");
                return;
            }
    });
    if (bad.load()) return fail(QXA_E_INVALID, why);
    parallel_for(tp.n_shared, [&](int64_t a, int64_t b) {
        for (int64_t k = a; k < b && !bad.load(); ++k) {
            const int32_t u = tp.fix_target[k], m = tp.fix_mirror[k];
            if (k > 0 && u <= tp.fix_target[k - 1]) return flag("tile plan: fix-up not sorted");
            if (u < 0 || u >= nnz || m < 0 || m >= nnz || hp.mirror[u] != uint32_t(m))
                return flag("tile plan: bad fix-up slot");
            if (tp.part_ptr[k + 1] <= tp.part_ptr[k]) return flag("tile plan: shared slot without partials");
            uint64_t acc = 0;
            for (int64_t q = tp.part_ptr[k]; q < tp.part_ptr[k + 1]; ++q) acc += part[q];
            if (!write_once(slot_ws[u])) return flag("tile plan: fix-up slot written twice");
            if (m != u && !write_once(slot_ws[m])) return flag("tile plan: fix-up mirror written twice");
            if (acc != expected(u) || (m != u && acc != expected(m)))
                return flag("tile plan: slot sum differs from the element entries");
        }
    });
    if (bad.load()) return fail(QXA_E_INVALID, why);
    std::atomic<bool> unwritten{false};
    parallel_for(nnz, [&](int64_t a, int64_t b) {
        for (int64_t u = a; u < b; ++u)
            if (slot_ws[u] != 1) unwritten = true;
    });
    if (unwritten) return fail(QXA_E_INVALID, "tile plan: CSR slot not written exactly once");
    return QXA_OK;
}

void tile_plan_stats(const TilePlan &tp, qxa_plan_info &o)
{
    o.n_tiles = tp.n_tiles;
    o.n_shared = tp.n_shared;
    o.n_partials = tp.n_partials;
    o.n_outputs = tp.n_outputs;
    o.n_units = tp.rec_ptr.empty() ? 0 : tp.rec_ptr.back();
    o.n_pair_units = 0;
    for (int64_t t = 0; t < tp.n_tiles; ++t) o.n_pair_units += tp.rec_mid[t] - tp.rec_ptr[t];
    o.n_chains = tp.chain_ptr.empty() ? 0 : int64_t(tp.chain_ptr.size()) - 1;
    o.n_carry_reads = tp.n_carry_reads;
    o.n_fix_slots = 0;
    for (size_t k = 0; k < tp.fix_target.size(); ++k) o.n_fix_slots += tp.fix_mirror[k] != tp.fix_target[k] ? 2 : 1;
    o.n_ext_units = tp.n_ext_units;
    o.n_empty_units = tp.n_empty_units;
    o.carry_cap = tp.carry_cap;
    o.carry_used = tp.carry_used;
}

}  // namespace qxa

// Kernelize: the dynamic program over ordered kernel sets of section "Circuit
// Kernelization" (Algorithm alg:dp; the kernel constraint of weak convexity
// and monotonicity), with the extensible-qubit bookkeeping of section
// "Reducing Size of DP State" (Algorithm alg:extensible), the two kernel
// types of section "Cost Function in Kernelize", and the appendix's
// optimisations as options: attaching one-qubit gates, subsumption, packing
// of adjacent kernels and pruning at T states.
//
// DP state before unit u: the closed kernels (final order) and the ordered
// set KS of open kernels, each with its type, qubit set Q, LDS need set, the
// extensible set E (kAll = every qubit), its LDS gate-cost sum and the set I
// of the commuting lift below.  Two states whose open kernels agree in
// (type, Q, need, E, I) have the same futures, so only the cheaper one stays
// (cost, kernel count, first made).
// Transitions for unit u:
//   * join an open kernel K whose E holds u's qubits and whose type stays
//     feasible; K stays in place when E != kAll (monotonicity applies) and
//     moves to the end of KS otherwise;
//   * open a new kernel {u} after closing any prefix of KS; it goes last.
// Then every other open kernel's E follows alg:extensible.  At the end the
// open kernels are closed in KS order.
//
// Commuting lift (QK_DP_COMMUTE, the appendix's insular qubits): in the
// intersect test of alg:extensible a shared qubit that is insular to the new
// unit and to every gate of the other kernel is ignored (such gates commute).
// Kernels can then pass each other with gates out of input order, so the
// ignored qubits are recorded in I on both kernels for their lifetime, and a
// unit joins a kernel in place only if it is insular on all of that kernel's
// I; without this record a later in-place join could overtake a gate it does
// not commute with.  Kernel membership and closed kernels
// are persistent linked lists, so a state copies only its open-kernel
// records.
#include <algorithm>
#include <unordered_map>

#include "plan.hpp"

namespace qk {

namespace {

constexpr uint64_t kAll = ~0ull;
constexpr int64_t kInfCost = int64_t(1) << 62;

struct DKer {
    int type;
    uint64_t q, need, ext;
    int64_t lsum;
    int32_t units;   // head of this kernel's unit list (most recent first)
    uint64_t ins;    // qubits the commuting lift ignored against other kernels
};

struct DState {
    int64_t v;       // total cost with every open kernel priced as it stands
    int64_t nk;      // kernels, closed + open
    int64_t ncl;     // closed kernels
    int32_t closed;  // head of the closed list (most recent first)
    uint32_t off, len;   // open kernels in the arena
};

struct UNode { int32_t unit, prev; };
struct CNode { int type; int32_t units; int64_t cost; int32_t prev; };

struct Unit {
    std::vector<int64_t> gates;   // canonical gate indices, execution order
    uint64_t q, need;
    int64_t lcost;
};

int pc(uint64_t x) { return __builtin_popcountll(x); }

struct Ctx {
    const qk_kopts& ko;
    const qk_cost_tables& tab;
    uint64_t lowmask;
    std::vector<UNode> un;
    std::vector<CNode> cn;

    int64_t cost(const DKer& K) const
    {
        return K.type == QK_KERNEL_FUSED ? tab.fused_ps[pc(K.q)] : tab.lds_alpha_ps + K.lsum;
    }
    bool feasible(int type, uint64_t q, uint64_t need) const
    {
        if (type == QK_KERNEL_FUSED)
            return ko.allow_fused && pc(q) <= ko.k_max && (ko.local_qubits <= 0 || ko.local_qubits >= 64 ||
                                                            (q >> ko.local_qubits) == 0);
        return ko.allow_lds && pc(need | lowmask) <= ko.m_max;
    }
    int32_t push_unit(int32_t unit, int32_t prev)
    {
        un.push_back({unit, prev});
        return (int32_t)un.size() - 1;
    }
    // list b appended after list a (both most-recent-first): copies b's nodes
    int32_t concat_units(int32_t a, int32_t b)
    {
        std::vector<int32_t> items;
        for (int32_t x = b; x >= 0; x = un[x].prev) items.push_back(un[x].unit);
        int32_t h = a;
        for (size_t t = items.size(); t-- > 0;) h = push_unit(items[t], h);
        return h;
    }
    // post-processing: merge each open kernel into the previous one of the
    // same type when the merged kernel is feasible and costs no more
    void pack(const DKer* open, uint32_t len, std::vector<DKer>& out)
    {
        out.clear();
        for (uint32_t i = 0; i < len; ++i) {
            const DKer& K = open[i];
            if (!out.empty() && out.back().type == K.type) {
                const DKer& P = out.back();
                DKer M{K.type, P.q | K.q, P.need | K.need, kAll, P.lsum + K.lsum, -1, 0};
                if (feasible(M.type, M.q, M.need) && cost(M) <= cost(P) + cost(K)) {
                    M.units = concat_units(P.units, K.units);
                    out.back() = M;
                    continue;
                }
            }
            out.push_back(K);
        }
    }
    // packed cost (units lists not built): used for pruning and the final pick
    int64_t packed_cost(const DKer* open, uint32_t len, int64_t* nout)
    {
        int64_t tot = 0, cnt = 0;
        bool have = false;
        DKer P{};
        for (uint32_t i = 0; i < len; ++i) {
            const DKer& K = open[i];
            if (have && P.type == K.type) {
                DKer M{K.type, P.q | K.q, P.need | K.need, kAll, P.lsum + K.lsum, -1, 0};
                if (feasible(M.type, M.q, M.need) && cost(M) <= cost(P) + cost(K)) {
                    P = M;
                    continue;
                }
            }
            if (have) { tot += cost(P); ++cnt; }
            P = K;
            have = true;
        }
        if (have) { tot += cost(P); ++cnt; }
        *nout = cnt;
        return tot;
    }
};

// alg:extensible for every open kernel but index `skip`, after a unit with
// qubits uq; with `commute`, shared qubits insular to the unit (outside its
// need set und) and to the kernel are ignored and recorded on both kernels
void update_others(DKer* ks, uint32_t len, uint32_t skip, uint64_t uq, uint64_t und, bool commute)
{
    uint64_t mine = 0;
    for (uint32_t j = 0; j < len; ++j) {
        if (j == skip) continue;
        DKer& K = ks[j];
        if (K.ext == kAll) {
            const uint64_t shared = uq & K.q;
            const uint64_t ign = commute ? shared & ~und & ~K.need : 0;
            if (shared & ~ign) {
                K.ext = K.q & ~uq;
            } else {
                K.ins |= ign;
                mine |= ign;
            }
        } else {
            K.ext &= ~uq;
        }
    }
    ks[skip].ins |= mine;
}

struct KeyHash {
    const std::vector<DKer>* arena;
    size_t operator()(const std::pair<uint32_t, uint32_t>& k) const
    {
        uint64_t h = 1469598103934665603ull ^ k.second;
        for (uint32_t i = 0; i < k.second; ++i) {
            const DKer& K = (*arena)[k.first + i];
            for (uint64_t w : {(uint64_t)K.type, K.q, K.need, K.ext, K.ins}) {
                h ^= w + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
            }
        }
        return (size_t)h;
    }
};
struct KeyEq {
    const std::vector<DKer>* arena;
    bool operator()(const std::pair<uint32_t, uint32_t>& a, const std::pair<uint32_t, uint32_t>& b) const
    {
        if (a.second != b.second) return false;
        for (uint32_t i = 0; i < a.second; ++i) {
            const DKer& x = (*arena)[a.first + i];
            const DKer& y = (*arena)[b.first + i];
            if (x.type != y.type || x.q != y.q || x.need != y.need || x.ext != y.ext || x.ins != y.ins)
                return false;
        }
        return true;
    }
};

// Units: a gate, or (attach_1q) a multi-qubit gate with the one-qubit gates
// attached to it: each one-qubit gate joins the next multi-qubit gate on its
// qubit, else the previous one; one-qubit gates on a qubit no multi-qubit gate
// touches form one unit at the position of their first gate.
void make_units(const std::vector<CGate>& G, const qk_kopts& ko, bool attach, std::vector<Unit>& units)
{
    const int64_t m = (int64_t)G.size();
    const bool insular = ko.insular != 0;
    std::vector<std::vector<int64_t>> order;
    if (!attach) {
        for (int64_t i = 0; i < m; ++i) order.push_back({i});
    } else {
        std::vector<int64_t> nxt(m, -1), prv(m, -1), last(kMaxQubits, -1), next(kMaxQubits, -1);
        for (int64_t i = 0; i < m; ++i) {
            if (G[i].nq >= 2) for (int t = 0; t < G[i].nq; ++t) last[G[i].q[t]] = i;
            else prv[i] = last[G[i].q[0]];
        }
        for (int64_t i = m - 1; i >= 0; --i) {
            if (G[i].nq >= 2) for (int t = 0; t < G[i].nq; ++t) next[G[i].q[t]] = i;
            else nxt[i] = next[G[i].q[0]];
        }
        std::vector<std::vector<int64_t>> before(m), after(m), lone(kMaxQubits);
        for (int64_t i = 0; i < m; ++i) {
            if (G[i].nq >= 2) continue;
            if (nxt[i] >= 0) before[nxt[i]].push_back(i);
            else if (prv[i] >= 0) after[prv[i]].push_back(i);
            else lone[G[i].q[0]].push_back(i);
        }
        for (int64_t i = 0; i < m; ++i) {
            if (G[i].nq >= 2) {
                std::vector<int64_t> u = before[i];
                u.push_back(i);
                u.insert(u.end(), after[i].begin(), after[i].end());
                order.push_back(u);
            } else if (nxt[i] < 0 && prv[i] < 0 && lone[G[i].q[0]][0] == i) {
                order.push_back(lone[G[i].q[0]]);
            }
        }
    }
    units.clear();
    for (auto& gi : order) {
        Unit u{gi, 0, 0, 0};
        for (int64_t g : gi) {
            for (int t = 0; t < G[g].nq; ++t) u.q |= 1ull << G[g].q[t];
            u.need |= need_mask(G[g], insular);
        }
        units.push_back(std::move(u));
    }
}

}  // namespace

int kernelize_dp(const std::vector<CGate>& G, const qk_kopts& ko, const qk_cost_tables& tab,
                 std::vector<int64_t>& order, std::vector<DPKernel>& kernels, int64_t& total)
{
    order.clear();
    kernels.clear();
    total = 0;
    if (G.empty()) return QK_OK;
    const uint32_t flags = (uint32_t)ko.dp_flags;
    const bool attach = flags & QK_DP_ATTACH_1Q, subsume = flags & QK_DP_SUBSUME, packing = flags & QK_DP_PACK,
               fork_fused = flags & QK_DP_FUSED, commute = flags & QK_DP_COMMUTE;
    const int64_t T = ko.dp_prune;
    std::vector<Unit> units;
    make_units(G, ko, attach, units);
    for (Unit& u : units) {
        u.lcost = 0;
        for (int64_t g : u.gates) u.lcost += tab.lds_gate_ps[gate_class(G[g].kind)];
    }
    Ctx C{ko, tab, (1ull << ko.ell) - 1, {}, {}};
    C.un.reserve(1 << 16);

    std::vector<DState> cur{{0, 0, 0, -1, 0, 0}}, nxt;
    std::vector<DKer> arena, narena;
    std::vector<DKer> tmp, pk;
    constexpr size_t kStateCap = size_t(1) << 22;

    for (size_t ui = 0; ui < units.size(); ++ui) {
        const Unit& U = units[ui];
        if (T > 0 && (int64_t)cur.size() >= T) {
            // pruning: keep the T/2 states of lowest packed cost
            std::vector<std::tuple<int64_t, int64_t, uint32_t>> sc;
            sc.reserve(cur.size());
            for (uint32_t s = 0; s < cur.size(); ++s) {
                const DState& S = cur[s];
                int64_t pv = S.v, npk = S.len;
                if (packing) {
                    int64_t openc = 0;
                    for (uint32_t j = 0; j < S.len; ++j) openc += C.cost(arena[S.off + j]);
                    pv = S.v - openc + C.packed_cost(arena.data() + S.off, S.len, &npk);
                }
                sc.emplace_back(pv, S.ncl + npk, s);
            }
            std::sort(sc.begin(), sc.end());
            sc.resize((size_t)(T / 2));
            std::sort(sc.begin(), sc.end(), [](const auto& a, const auto& b) { return std::get<2>(a) < std::get<2>(b); });
            std::vector<DState> kept;
            kept.reserve(sc.size());
            for (auto& e : sc) kept.push_back(cur[std::get<2>(e)]);
            cur.swap(kept);
        }
        nxt.clear();
        narena.clear();
        std::unordered_map<std::pair<uint32_t, uint32_t>, uint32_t, KeyHash, KeyEq> idx(
            cur.size() * 4 + 16, KeyHash{&narena}, KeyEq{&narena});
        auto offer = [&](int64_t v, int64_t nk, int64_t ncl, int32_t closed, const std::vector<DKer>& open) {
            const uint32_t off = (uint32_t)narena.size(), len = (uint32_t)open.size();
            narena.insert(narena.end(), open.begin(), open.end());
            auto it = idx.find({off, len});
            if (it == idx.end()) {
                idx.emplace(std::make_pair(off, len), (uint32_t)nxt.size());
                nxt.push_back({v, nk, ncl, closed, off, len});
                return;
            }
            DState& E = nxt[it->second];
            if (v < E.v || (v == E.v && nk < E.nk)) {
                // same key: overwrite the stored kernels (same descriptors,
                // other members) and the state's totals in place
                std::copy(open.begin(), open.end(), narena.begin() + E.off);
                E.v = v; E.nk = nk; E.ncl = ncl; E.closed = closed;
            }
            narena.resize(off);
        };
        for (const DState& S : cur) {
            const DKer* ks = arena.data() + S.off;   // len may be 0 at the end of the arena
            std::vector<uint32_t> cands;
            for (uint32_t j = 0; j < S.len; ++j) {
                const DKer& K = ks[j];
                if (K.ext != kAll && ((U.q & ~K.ext) || (U.need & K.ins))) continue;
                if (!C.feasible(K.type, K.q | U.q, K.need | U.need)) continue;
                cands.push_back(j);
            }
            int64_t sub = -1;
            if (subsume)
                for (uint32_t j : cands)
                    if ((U.q & ~ks[j].q) == 0 || (ks[j].q & ~U.q) == 0) { sub = j; break; }
            auto add_to = [&](uint32_t j) {
                const DKer& K = ks[j];
                DKer K2{K.type, K.q | U.q, K.need | U.need, K.ext, K.lsum + U.lcost,
                        C.push_unit((int32_t)ui, K.units), K.ins};
                const int64_t dv = C.cost(K2) - C.cost(K);
                tmp.assign(ks, ks + S.len);
                if (K.ext == kAll) {
                    tmp.erase(tmp.begin() + j);
                    tmp.push_back(K2);
                    update_others(tmp.data(), (uint32_t)tmp.size(), (uint32_t)tmp.size() - 1, U.q, U.need, commute);
                } else {
                    tmp[j] = K2;
                    update_others(tmp.data(), (uint32_t)tmp.size(), j, U.q, U.need, commute);
                }
                offer(S.v + dv, S.nk, S.ncl, S.closed, tmp);
            };
            if (sub >= 0) {
                add_to((uint32_t)sub);
                continue;
            }
            for (uint32_t j : cands) add_to(j);
            for (int t : {QK_KERNEL_FUSED, QK_KERNEL_LDS}) {
                if ((t == QK_KERNEL_FUSED && !fork_fused) || !C.feasible(t, U.q, U.need)) continue;
                DKer Kn{t, U.q, U.need, kAll, U.lcost, C.push_unit((int32_t)ui, -1), 0};
                const int64_t cnew = C.cost(Kn);
                int32_t closed = S.closed;
                for (uint32_t p = 0; p <= S.len; ++p) {
                    if (p > 0) {
                        const DKer& Kc = ks[p - 1];
                        C.cn.push_back({Kc.type, Kc.units, C.cost(Kc), closed});
                        closed = (int32_t)C.cn.size() - 1;
                    }
                    tmp.assign(ks + p, ks + S.len);
                    tmp.push_back(Kn);
                    update_others(tmp.data(), (uint32_t)tmp.size(), (uint32_t)tmp.size() - 1, U.q, U.need, commute);
                    offer(S.v + cnew, S.nk + 1, S.ncl + p, closed, tmp);
                }
            }
        }
        if (nxt.empty()) return fail(QK_EINVAL, "kernelize: gate unit " + std::to_string(ui) + " fits no kernel type");
        if (nxt.size() > kStateCap)
            return fail(QK_EUNSUPPORTED, "kernelize: more than 2^22 DP states (set dp_prune)");
        cur.swap(nxt);
        arena.swap(narena);
    }
    // final pick: closed + (packed) open kernels, lowest (cost, count, index)
    int64_t best_tot = kInfCost, best_n = 0;
    int64_t best_s = -1;
    for (uint32_t s = 0; s < cur.size(); ++s) {
        const DState& S = cur[s];
        int64_t closed_cost = 0;
        for (int32_t c = S.closed; c >= 0; c = C.cn[c].prev) closed_cost += C.cn[c].cost;
        int64_t npk = S.len, oc = 0;
        if (packing) oc = C.packed_cost(arena.data() + S.off, S.len, &npk);
        else for (uint32_t j = 0; j < S.len; ++j) oc += C.cost(arena[S.off + j]);
        const int64_t tot = closed_cost + oc, nks = S.ncl + npk;
        if (tot < best_tot || (tot == best_tot && nks < best_n)) {
            best_tot = tot;
            best_n = nks;
            best_s = s;
        }
    }
    const DState& B = cur[best_s];
    std::vector<const CNode*> cl;
    for (int32_t c = B.closed; c >= 0; c = C.cn[c].prev) cl.push_back(&C.cn[c]);
    std::reverse(cl.begin(), cl.end());
    std::vector<std::pair<int, int32_t>> seq;   // (type, units head)
    std::vector<int64_t> costs;
    for (const CNode* c : cl) { seq.push_back({c->type, c->units}); costs.push_back(c->cost); }
    if (packing) C.pack(arena.data() + B.off, B.len, pk);
    else pk.assign(arena.begin() + B.off, arena.begin() + B.off + B.len);
    for (const DKer& K : pk) { seq.push_back({K.type, K.units}); costs.push_back(C.cost(K)); }
    for (size_t k = 0; k < seq.size(); ++k) {
        std::vector<int32_t> us;
        for (int32_t x = seq[k].second; x >= 0; x = C.un[x].prev) us.push_back(C.un[x].unit);
        std::reverse(us.begin(), us.end());
        DPKernel dk{seq[k].first, (int64_t)order.size(), 0, costs[k]};
        for (int32_t u : us) order.insert(order.end(), units[u].gates.begin(), units[u].gates.end());
        dk.end = (int64_t)order.size();
        kernels.push_back(dk);
    }
    total = best_tot;
    return QK_OK;
}

}  // namespace qk

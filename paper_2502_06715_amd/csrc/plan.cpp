// Host-side planning: query validation, the per-level Generic Join plan with the
// lifted intersections of Section 6.1, and the order/share decision of
// Sections 6.2-6.3.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <functional>
#include <numeric>

#include "hc_internal.h"

namespace hc {

void validate_query(const hc_query* q, int max_arity) {
    int covered[kMaxVars] = {0};
    int off = 0;
    for (int j = 0; j < q->n_atoms; ++j) {
        const int k = q->atom_arity[j];
        HC_REQUIRE(k >= 1 && k <= 4, HC_ERR_INVALID, "atom arity must be 1..4");
        HC_REQUIRE(k <= max_arity, HC_ERR_UNSUPPORTED, "atoms of arity > " + std::to_string(max_arity) +
                                                            " are not supported by the join engine");
        for (int c = 0; c < k; ++c) {
            const int v = q->atom_vars[off + c];
            HC_REQUIRE(v >= 0 && v < q->n_vars, HC_ERR_INVALID, "atom variable out of range");
            for (int c2 = 0; c2 < c; ++c2)
                HC_REQUIRE(q->atom_vars[off + c2] != v, HC_ERR_UNSUPPORTED, "variable repeated inside one atom");
            covered[v] = 1;
        }
        off += k;
    }
    for (int v = 0; v < q->n_vars; ++v)
        HC_REQUIRE(covered[v], HC_ERR_INVALID, "variable " + std::to_string(v) + " occurs in no atom");
    if (q->var_lo)
        for (int v = 0; v < q->n_vars; ++v)
            HC_REQUIRE(q->var_lo[v] <= q->var_hi[v], HC_ERR_INVALID, "var_lo > var_hi");
}

static void check_order(const hc_query* q, const int32_t* order) {
    int seen[kMaxVars] = {0};
    for (int i = 0; i < q->n_vars; ++i) {
        HC_REQUIRE(order[i] >= 0 && order[i] < q->n_vars && !seen[order[i]], HC_ERR_INVALID,
                   "var_order must be a permutation of the variables");
        seen[order[i]] = 1;
    }
}

// Generic Join plan.  Level i (0-based) binds order[i].  Each atom holding the
// variable contributes one operand: its top level V0 when the variable is the
// atom's first in the order, else the child list of the atom's entry bound at
// the level of its first variable.  Call d the level at which that operand's
// dependency is bound (-1 for V0).  Operands with d < i-1 do not change while
// level i-1 iterates; when two or more exist, their intersection is lifted to
// frontier F_{max d + 1} (computed once per binding of levels <= max d) and
// consumed at level i as one temporary operand (Section 6.1).
Plan compile_plan(const hc_query* q, const int32_t* order, bool rewrite, int min_lift) {
    validate_query(q, 4);
    check_order(q, order);
    Plan p;
    p.n_vars = q->n_vars;
    p.n_atoms = q->n_atoms;
    for (int i = 0; i < q->n_vars; ++i) {
        p.order[i] = order[i];
        p.pos[order[i]] = i;
    }
    int off = 0;
    for (int j = 0; j < q->n_atoms; ++j) {
        const int k = q->atom_arity[j];
        p.atom_arity[j] = k;
        // CoCo levels of an atom follow the variable order (Section 4)
        int lv[4];
        for (int c = 0; c < k; ++c) lv[c] = q->atom_vars[off + c];
        for (int x = 1; x < k; ++x)
            for (int y = x; y > 0 && p.pos[lv[y]] < p.pos[lv[y - 1]]; --y) std::swap(lv[y], lv[y - 1]);
        for (int r = 0; r < 4; ++r) p.atom_lvl_var[j][r] = r < k ? lv[r] : -1;
        p.atom_first[j] = lv[0];
        p.atom_second[j] = k > 1 ? lv[1] : -1;
        off += k;
    }
    p.n_groups = 0;
    for (int i = 0; i < q->n_vars; ++i) {
        const int x = order[i];
        PlanOp ops[kMaxAtoms];
        int dep[kMaxAtoms];
        int n = 0;
        for (int j = 0; j < q->n_atoms; ++j) {
            for (int r = 0; r < p.atom_arity[j]; ++r) {
                if (p.atom_lvl_var[j][r] != x) continue;
                if (r == 0) {
                    ops[n] = PlanOp{OP_V0, j, -1, 0};
                    dep[n++] = -1;
                } else {   // children of the atom's node at level r-1, bound at its parent's level
                    ops[n] = PlanOp{OP_CHILD, j, -1, r};
                    dep[n++] = p.pos[p.atom_lvl_var[j][r - 1]];
                }
            }
        }
        HC_REQUIRE(n <= kMaxOps, HC_ERR_UNSUPPORTED, "more than 8 atoms share one variable");
        int n_low = 0, max_low = -1;
        for (int t = 0; t < n; ++t)
            if (dep[t] < i - 1) {
                ++n_low;
                max_low = std::max(max_low, dep[t]);
            }
        PlanLevel& L = p.levels[i];
        L.var = x;
        L.n_ops = 0;
        if (rewrite && n_low >= 2 && max_low + 1 >= min_lift) {
            HC_REQUIRE(p.n_groups < kMaxGroups, HC_ERR_UNSUPPORTED, "too many lifted intersections");
            PlanGroup& g = p.groups[p.n_groups];
            g.var = x;
            g.consumer = i;
            g.lift = max_low + 1;
            g.n_ops = 0;
            for (int t = 0; t < n; ++t)
                if (dep[t] < i - 1) g.ops[g.n_ops++] = ops[t];
                else L.ops[L.n_ops++] = ops[t];
            L.ops[L.n_ops++] = PlanOp{OP_TMP, -1, p.n_groups, 0};
            ++p.n_groups;
        } else {
            for (int t = 0; t < n; ++t) L.ops[L.n_ops++] = ops[t];
        }
        L.n_new_nodes = 0;
        for (int j = 0; j < q->n_atoms; ++j)
            for (int r = 0; r + 1 < p.atom_arity[j]; ++r)
                if (p.atom_lvl_var[j][r] == x) L.new_node_atom[L.n_new_nodes++] = j;
    }
    return p;
}

std::string describe_plan(const Plan& p) {
    std::string s = "{\"order\": [";
    for (int i = 0; i < p.n_vars; ++i) s += (i ? ", " : "") + std::to_string(p.order[i]);
    s += "], \"levels\": [";
    auto op_str = [&](const PlanOp& o) {
        const char* k = o.kind == OP_V0 ? "V0" : o.kind == OP_CHILD ? "CHILD" : "TMP";
        std::string t = std::string("{\"kind\": \"") + k + "\"";
        if (o.kind == OP_TMP) t += ", \"group\": " + std::to_string(o.group);
        else t += ", \"atom\": " + std::to_string(o.atom);
        return t + "}";
    };
    for (int i = 0; i < p.n_vars; ++i) {
        const PlanLevel& L = p.levels[i];
        s += (i ? ", " : "");
        s += "{\"level\": " + std::to_string(i + 1) + ", \"var\": " + std::to_string(L.var) + ", \"ops\": [";
        for (int t = 0; t < L.n_ops; ++t) s += (t ? ", " : "") + op_str(L.ops[t]);
        s += "], \"lift\": ";
        int g = -1;
        for (int t = 0; t < p.n_groups; ++t)
            if (p.groups[t].consumer == i) g = t;
        if (g < 0) {
            s += "null";
        } else {
            // lift level in the paper's numbering: 0 = before the outermost loop
            std::vector<int> at;
            for (int t = 0; t < p.groups[g].n_ops; ++t) at.push_back(p.groups[g].ops[t].atom);
            std::sort(at.begin(), at.end());
            s += "[" + std::to_string(p.groups[g].lift) + ", [";
            for (size_t t = 0; t < at.size(); ++t) s += (t ? ", " : "") + std::to_string(at[t]);
            s += "]]";
        }
        s += "}";
    }
    return s + "]}";
}

// ---------------------------------------------------------------- cost model
// Per-level cost (Section 6.2): |S| * min N * log2(1 + max N / min N) for one
// binding, summed over the bindings of the prefix via the Lemma's bound with
// the averages of the worked example: avg |R[x].Y| = |R| / |R.X|.  The number
// of prefix bindings is bounded by chaining the smallest operand of every
// level (the intersection is never larger than its smallest operand).
// Lifted operands are charged at their lift level and replaced at the consumer
// level by the temporary result, whose size is the smallest lifted operand.
struct LevelCost {
    double C[kMaxVars];
    double total;
};

// Pessimistic variant (HC_PESSIMISTIC, an upper bound in place of the averages'
// chain, in the role of the estimator the paper cites): the bindings of the prefix
// X_1..X_i are at most those of X_1..X_{i-1} times the longest list of the level's
// shortest operand, and at most |R_j| times the domains of the prefix variables
// outside R_j for every atom R_j whose variables all lie in the prefix; Sum min N
// of the Lemma is that bound, and the ratio inside the logarithm keeps the
// averages of the worked example.
static LevelCost level_costs(const hc_query* q, const std::vector<AtomStats>& st, const Plan& p,
                             bool pessimistic = false) {
    LevelCost lc{};
    // column index of a variable inside atom j
    auto col_of = [&](int j, int v) {
        int off = 0;
        for (int t = 0; t < j; ++t) off += q->atom_arity[t];
        for (int c = 0; c < q->atom_arity[j]; ++c)
            if (q->atom_vars[off + c] == v) return c;
        return 0;
    };
    auto avg_n = [&](const PlanOp& o, int var) {
        const AtomStats& a = st[o.atom];
        if (o.kind == OP_V0) return std::max(1.0, a.distinct[col_of(o.atom, var)]);
        // children per node of level lvl-1: rows over the distinct prefixes of length lvl
        double parents = 1.0;
        for (int r = 0; r < o.lvl; ++r) parents *= std::max(1.0, a.distinct[col_of(o.atom, p.atom_lvl_var[o.atom][r])]);
        return std::max(1.0, a.rows / std::max(1.0, std::min(parents, a.rows)));
    };
    auto cost_of = [](int nops, double bind, double mn, double mx) {
        if (nops <= 1) return bind * mn;
        return (double)nops * bind * mn * std::log2(1.0 + mx / mn);
    };
    // longest list an operand can offer (pessimistic estimator)
    auto max_n = [&](const PlanOp& o, int var) {
        const AtomStats& a = st[o.atom];
        if (o.kind == OP_V0) return std::max(1.0, a.distinct[col_of(o.atom, var)]);
        const double md = a.maxdeg[o.lvl - 1];
        return md > 0 ? md : std::max(1.0, a.rows);
    };
    std::vector<double> dom(p.n_vars, 1e300);
    {
        int off = 0;
        for (int j = 0; j < q->n_atoms; ++j) {
            for (int c = 0; c < q->atom_arity[j]; ++c)
                dom[q->atom_vars[off + c]] = std::min(dom[q->atom_vars[off + c]], std::max(1.0, st[j].distinct[c]));
            off += q->atom_arity[j];
        }
    }
    auto prefix_cap = [&](int i) {   // bound on |Q(X_sigma(1..i+1))| from whole atoms inside the prefix
        double cap = 1e300;
        for (int j = 0; j < q->n_atoms; ++j) {
            bool inside = true;
            for (int r = 0; r < p.atom_arity[j]; ++r) inside = inside && p.pos[p.atom_lvl_var[j][r]] <= i;
            if (!inside) continue;
            double b = std::max(1.0, st[j].rows);
            for (int t = 0; t <= i; ++t) {
                bool in_atom = false;
                for (int r = 0; r < p.atom_arity[j]; ++r) in_atom = in_atom || p.atom_lvl_var[j][r] == p.order[t];
                if (!in_atom) b *= dom[p.order[t]];
            }
            cap = std::min(cap, b);
        }
        return cap;
    };
    double bind = 1.0;   // bindings of the prefix at the current level
    double tmp_size[kMaxGroups];
    for (int i = 0; i < p.n_vars; ++i) {
        const PlanLevel& L = p.levels[i];
        // groups lifted to frontier F_i are computed here
        double extra = 0.0;
        for (int g = 0; g < p.n_groups; ++g) {
            if (p.groups[g].lift != i) continue;
            double mn = 1e300, mx = 0;
            for (int t = 0; t < p.groups[g].n_ops; ++t) {
                const double n = avg_n(p.groups[g].ops[t], p.groups[g].var);
                mn = std::min(mn, n);
                mx = std::max(mx, n);
            }
            tmp_size[g] = mn;
            extra += cost_of(p.groups[g].n_ops, bind, mn, mx);
        }
        double mn = 1e300, mx = 0, mn_max = 1e300;
        for (int t = 0; t < L.n_ops; ++t) {
            const double n = L.ops[t].kind == OP_TMP ? tmp_size[L.ops[t].group] : avg_n(L.ops[t], L.var);
            mn = std::min(mn, n);
            mx = std::max(mx, n);
            if (L.ops[t].kind != OP_TMP) mn_max = std::min(mn_max, max_n(L.ops[t], L.var));
        }
        if (!pessimistic) {
            // lifted work is charged to the level where it runs
            lc.C[i] = cost_of(L.n_ops, bind, mn, mx) + extra;
            bind = bind * mn;
        } else {
            const double next = std::min(bind * std::min(mn_max, 1e300), prefix_cap(i));   // Sum min N bound
            lc.C[i] = (L.n_ops <= 1 ? next : (double)L.n_ops * next * std::log2(1.0 + mx / mn)) + extra;
            bind = next;
        }
    }
    lc.total = 0;
    for (int i = 0; i < p.n_vars; ++i) lc.total += lc.C[i];
    return lc;
}

// Eq. (total cost): every level's cost is repeated by the product of the shares
// of the variables bound after it (cells that differ only in later coordinates
// rediscover the same outer bindings).
static double share_cost(const Plan& p, const LevelCost& lc, const int* k_of_var) {
    double tot = 0;
    for (int i = 0; i < p.n_vars; ++i) {
        double rep = 1;
        for (int j = i + 1; j < p.n_vars; ++j) rep *= std::ldexp(1.0, k_of_var[p.order[j]]);
        tot += rep * lc.C[i];
    }
    return tot;
}

// |Dom(X_v)|: the fewest distinct values any atom holding v offers; key bits bound the share
static void domains(const hc_query* q, const std::vector<AtomStats>& st, std::vector<double>& dom,
                    std::vector<int>& maxbits) {
    dom.assign(q->n_vars, 1e300);
    maxbits.assign(q->n_vars, 32);
    int off = 0;
    for (int j = 0; j < q->n_atoms; ++j) {
        for (int c = 0; c < q->atom_arity[j]; ++c) {
            const int v = q->atom_vars[off + c];
            dom[v] = std::min(dom[v], st[j].distinct[c]);
            maxbits[v] = std::min(maxbits[v], st[j].dom_bits);
        }
        off += q->atom_arity[j];
    }
}

static bool share_feasible(const std::vector<int>& kv, const std::vector<double>& dom, const std::vector<int>& maxbits) {
    for (size_t v = 0; v < kv.size(); ++v) {
        if (kv[v] > maxbits[v]) return false;
        if (kv[v] > 0) {
            const double P = std::ldexp(1.0, kv[v]);
            if (dom[v] < 3.0 * P * std::log(P)) return false;
        }
    }
    return true;
}

// Joint search (HC_JOINT_SEARCH): every order and every share vector of the plan
// decision of Section 6.3; a vector is feasible when its Eq. (total cost) is at most
// twice the best unpartitioned cost over all orders and it passes the domain rule;
// the minimum evenness wins, then the lower cost, then the earlier order.
static void joint_search(const hc_query* q, const std::vector<AtomStats>& st, int K, uint32_t flags,
                         int32_t* order_out, int32_t* shares_out) {
    const int n = q->n_vars;
    const bool rewrite = !(flags & HC_NO_REWRITE);
    const bool pess = (flags & HC_PESSIMISTIC) != 0;
    std::vector<std::vector<int32_t>> orders;
    std::vector<Plan> plans;
    std::vector<LevelCost> costs;
    std::vector<int32_t> o(n);
    std::iota(o.begin(), o.end(), 0);
    double base = 1e308;
    do {
        orders.push_back(o);
        plans.push_back(compile_plan(q, o.data(), rewrite));
        costs.push_back(level_costs(q, st, plans.back(), pess));
        base = std::min(base, costs.back().total);
    } while (std::next_permutation(o.begin(), o.end()));
    std::vector<double> dom;
    std::vector<int> maxbits;
    domains(q, st, dom, maxbits);
    bool found = false, fb_found = false;
    double best_E = 1e308, best_c = 1e308, fb_c = 1e308;
    std::vector<int> best_k(n, 0), fb_k(n, 0), k(n, 0), kv(n, 0);
    size_t best_o = 0, fb_o = 0;
    for (size_t t = 0; t < orders.size(); ++t) {
        const Plan& p = plans[t];
        std::function<void(int, int)> rec = [&](int lvl, int left) {
            if (lvl < n - 1) {
                for (int x = 0; x <= left; ++x) {
                    k[lvl] = x;
                    rec(lvl + 1, left - x);
                }
                return;
            }
            k[lvl] = left;
            for (int i = 0; i < n; ++i) kv[p.order[i]] = k[i];
            if (!share_feasible(kv, dom, maxbits)) return;
            const double c = share_cost(p, costs[t], kv.data());
            if (c < fb_c) {
                fb_c = c;
                fb_k = kv;
                fb_o = t;
                fb_found = true;
            }
            if (c > 2.0 * base) return;
            double E = 0;
            for (int i = 0; i < n; ++i) E += std::ldexp(1.0, k[i]) * std::max(1.0 - (i + 1) / 100.0, 0.75);
            if (!found || E < best_E - 1e-9 || (std::fabs(E - best_E) <= 1e-9 && c < best_c * (1 - 1e-12))) {
                found = true;
                best_E = E;
                best_c = c;
                best_k = kv;
                best_o = t;
            }
        };
        rec(0, K);
    }
    const size_t ot = found ? best_o : fb_o;
    const std::vector<int>& pick = found ? best_k : (fb_found ? fb_k : std::vector<int>(n, 0));
    for (int i = 0; i < n; ++i) order_out[i] = orders[ot][i];
    for (int v = 0; v < n; ++v) shares_out[v] = pick[v];
}

double plan_cost(const hc_query* q, const std::vector<AtomStats>& st, const int32_t* order, const int32_t* shares,
                 uint32_t flags, double* per_level) {
    validate_query(q, 4);
    const Plan p = compile_plan(q, order, !(flags & HC_NO_REWRITE));
    const LevelCost lc = level_costs(q, st, p, (flags & HC_PESSIMISTIC) != 0);
    double tot = 0;
    for (int i = 0; i < p.n_vars; ++i) {
        double rep = 1;
        for (int j = i + 1; j < p.n_vars; ++j) rep *= std::ldexp(1.0, shares ? shares[p.order[j]] : 0);
        if (per_level) per_level[i] = rep * lc.C[i];
        tot += rep * lc.C[i];
    }
    return tot;
}

// HC_CACHE_SHARES: cheapest share vector (Eq. (total cost)) among those whose every
// atom's per-cell slice fits one XCD's L2; failing that, the smallest largest slice.
static void cache_shares(const hc_query* q, const std::vector<AtomStats>& st, const Plan& p, const LevelCost& lc,
                         int K, int32_t* shares_out) {
    constexpr double kL2 = 4.0 * 1024 * 1024;   // bytes of L2 per XCD
    const int n = q->n_vars;
    std::vector<double> dom;
    std::vector<int> maxbits;
    domains(q, st, dom, maxbits);
    std::vector<int> k(n, 0), kv(n, 0), best(n, 0);
    bool found = false, best_fits = false;
    double best_c = 1e308, best_slice = 1e308;
    std::function<void(int, int)> rec = [&](int lvl, int left) {
        if (lvl < n - 1) {
            for (int x = 0; x <= left; ++x) {
                k[lvl] = x;
                rec(lvl + 1, left - x);
            }
            return;
        }
        k[lvl] = left;
        for (int i = 0; i < n; ++i) kv[p.order[i]] = k[i];
        if (!share_feasible(kv, dom, maxbits)) return;
        double slice = 0;
        int off = 0;
        for (int j = 0; j < q->n_atoms; ++j) {
            int bits = 0;
            for (int c = 0; c < q->atom_arity[j]; ++c) bits += kv[q->atom_vars[off + c]];
            off += q->atom_arity[j];
            slice = std::max(slice, std::ldexp(4.0 * st[j].rows, -bits));
        }
        const double c = share_cost(p, lc, kv.data());
        const bool fits = slice <= kL2;
        bool better;
        if (!found) better = true;
        else if (fits != best_fits) better = fits;
        else if (fits) better = c < best_c * (1 - 1e-12);
        else better = slice < best_slice * (1 - 1e-12) || (slice <= best_slice * (1 + 1e-12) && c < best_c * (1 - 1e-12));
        if (better) {
            found = true;
            best_fits = fits;
            best_c = c;
            best_slice = slice;
            best = kv;
        }
    };
    rec(0, K);
    for (int v = 0; v < n; ++v) shares_out[v] = found ? best[v] : 0;
}

void choose_shares(const hc_query* q, const std::vector<AtomStats>& st, int K, uint32_t flags, int32_t* order_inout,
                   int32_t* shares_out) {
    const int n = q->n_vars;
    const bool rewrite = !(flags & HC_NO_REWRITE);
    const bool pess = (flags & HC_PESSIMISTIC) != 0;
    if ((flags & HC_JOINT_SEARCH) && !(flags & HC_KEEP_ORDER)) {
        joint_search(q, st, K, flags, order_inout, shares_out);
        return;
    }
    std::vector<int32_t> best_order(n);
    if (flags & HC_KEEP_ORDER) {
        check_order(q, order_inout);
        for (int i = 0; i < n; ++i) best_order[i] = order_inout[i];
    } else {
        // sigma* = argmin of the unpartitioned cost over all n! orders; ties: first in
        // lexicographic order.
        std::vector<int32_t> o(n);
        std::iota(o.begin(), o.end(), 0);
        double best = 1e308;
        do {
            Plan p = compile_plan(q, o.data(), rewrite);
            const double c = level_costs(q, st, p, pess).total;
            if (c < best * (1 - 1e-12)) {
                best = c;
                best_order = o;
            }
        } while (std::next_permutation(o.begin(), o.end()));
    }
    for (int i = 0; i < n; ++i) order_inout[i] = best_order[i];
    Plan p = compile_plan(q, best_order.data(), rewrite);
    const LevelCost lc = level_costs(q, st, p, pess);
    if (flags & HC_CACHE_SHARES) {
        cache_shares(q, st, p, lc, K, shares_out);
        return;
    }
    std::vector<double> dom;
    std::vector<int> maxbits;
    domains(q, st, dom, maxbits);
    // enumerate all power-of-two share vectors with sum k_v = K (shares by level)
    std::vector<int> k(n, 0), kv(n, 0), best_k(n, 0);
    double best_E = 1e308, best_cost = 1e308;
    bool found = false;
    double fb_cost = 1e308;
    std::vector<int> fb_k(n, 0);
    bool fb_found = false;
    const double base = lc.total;
    std::function<void(int, int)> rec = [&](int lvl, int left) {
        if (lvl == n - 1) {
            k[lvl] = left;
        } else {
            for (int t = 0; t <= left; ++t) {
                k[lvl] = t;
                rec(lvl + 1, left - t);
            }
            return;
        }
        for (int i = 0; i < n; ++i) kv[p.order[i]] = k[i];
        if (!share_feasible(kv, dom, maxbits)) return;
        const double c = share_cost(p, lc, kv.data());
        if (c < fb_cost) {
            fb_cost = c;
            fb_k = kv;
            fb_found = true;
        }
        if (c > 2.0 * base) return;
        double E = 0;
        for (int i = 0; i < n; ++i) E += std::ldexp(1.0, k[i]) * std::max(1.0 - (i + 1) / 100.0, 0.75);
        // ties: lower cost, then more shares on later variables
        bool better = false;
        if (!found || E < best_E - 1e-9) better = true;
        else if (std::fabs(E - best_E) <= 1e-9) {
            if (c < best_cost * (1 - 1e-12)) better = true;
            else if (std::fabs(c - best_cost) <= 1e-12 * best_cost) {
                for (int i = n - 1; i >= 0; --i) {
                    const int a = kv[p.order[i]], b = best_k[p.order[i]];
                    if (a != b) {
                        better = a > b;
                        break;
                    }
                }
            }
        }
        if (better) {
            found = true;
            best_E = E;
            best_cost = c;
            best_k = kv;
        }
    };
    rec(0, K);
    const std::vector<int>& pick = found ? best_k : (fb_found ? fb_k : std::vector<int>(n, 0));
    for (int v = 0; v < n; ++v) shares_out[v] = pick[v];
}

}  // namespace hc

// Bottom-up association-rule mining over binary items (Section 4.3), the
// whole level-wise search in the library:
//
//   level 1   item supports from the database marginals;
//   level 2   every pair support at once from the co-occurrence Gram
//             (fc_pairs, FP4 matrix cores);
//   level k   candidates joined from frequent (k-1)-itemsets that share their
//             first k-2 items, kept when every (k-1)-subset is frequent
//             (anti-monotonicity), counted in batches of single-assignment
//             queries Count(X_a = 1 AND ...) (fc_count_assignments: one path
//             of bit-vector intersections and a popcount each).
//
// An itemset S is frequent when Count(S)/m > minsup and a rule S - {X} => X
// is kept when Count(S)/Count(S - {X}) > minconf, both decided in binary64.
// Itemsets of a level are held sorted (lexicographic item ids), so every
// subset lookup is a binary search in the level below.
#include <algorithm>
#include <cstring>
#include <thread>
#include <vector>

#include "fc_internal.h"

struct fc_arm_result {
    // itemsets, level by level, lexicographic within a level
    std::vector<int32_t> set_items;
    std::vector<int64_t> set_off{0};
    std::vector<int64_t> set_count;
    // rules ordered by (antecedent, consequent) as tuples compare
    std::vector<int32_t> rule_items;
    std::vector<int64_t> rule_off{0};
    std::vector<int32_t> rule_cons;
    std::vector<double> rule_support, rule_conf;
};

namespace fc {
namespace {

// One level: n itemsets of k items each, sorted, with their counts.
struct Level {
    int32_t k = 0;
    std::vector<int32_t> items;  // n * k
    std::vector<int64_t> count;  // n
    int64_t size() const { return (int64_t)count.size(); }
    const int32_t *at(int64_t i) const { return items.data() + i * k; }
    // open-addressing index of the itemsets (built once the level is final)
    std::vector<int64_t> slot;  // itemset index, -1 empty
    uint64_t mask = 0;
    static uint64_t hash(const int32_t *s, int32_t k) {
        uint64_t h = 0x9E3779B97F4A7C15ull;
        for (int32_t t = 0; t < k; ++t) {
            h = (h ^ (uint32_t)s[t]) * 0xBF58476D1CE4E5B9ull;
            h ^= h >> 31;
        }
        return h;
    }
    void index() {
        uint64_t cap = 16;
        while (cap < 2 * (uint64_t)size()) cap <<= 1;
        slot.assign(cap, -1);
        mask = cap - 1;
        for (int64_t i = 0; i < size(); ++i) {
            uint64_t h = hash(at(i), k) & mask;
            while (slot[h] >= 0) h = (h + 1) & mask;
            slot[h] = i;
        }
    }
    // index of the itemset equal to s (k items), or -1
    int64_t find(const int32_t *s) const {
        for (uint64_t h = hash(s, k) & mask; slot[h] >= 0; h = (h + 1) & mask)
            if (std::equal(s, s + k, at(slot[h]))) return slot[h];
        return -1;
    }
};

bool frequent(int64_t count, int64_t m, double minsup) {
    return m > 0 && (double)count / (double)m > minsup;
}

// Apriori join of `prev` (sorted, indexed (k-1)-itemsets): pairs a < b of a
// block that shares the first k-2 items give prefix + {last_a, last_b}; a
// candidate is kept when each of its (k-1)-subsets that drops one of the
// prefix items is in `prev` (the two that drop a last item are the joined
// pair itself).  Rows a are split over host threads in contiguous ranges of
// equal pair counts (one block can hold most of the pairs); concatenating
// the ranges keeps the output lexicographic.
std::vector<int32_t> candidates(const Level &prev) {
    const int32_t k1 = prev.k, k = k1 + 1;
    const int64_t n = prev.size();
    std::vector<int64_t> bend((size_t)n), wsum((size_t)n + 1, 0);  // block end, pair prefix sums
    for (int64_t i = 0; i < n;) {
        int64_t j = i + 1;
        while (j < n && std::equal(prev.at(i), prev.at(i) + (k1 - 1), prev.at(j))) ++j;
        for (int64_t x = i; x < j; ++x) bend[(size_t)x] = j;
        i = j;
    }
    for (int64_t a = 0; a < n; ++a) wsum[(size_t)a + 1] = wsum[(size_t)a] + (bend[(size_t)a] - a - 1);
    const int64_t total = wsum[(size_t)n];
    unsigned hw = std::thread::hardware_concurrency();
    const int64_t T = std::max<int64_t>(
        1, std::min<int64_t>((int64_t)std::min(16u, hw ? hw : 1u), total / 8192 + 1));
    auto first_row = [&](int64_t t) {  // first row of range t
        if (t >= T) return n;
        return (int64_t)(std::lower_bound(wsum.begin(), wsum.end() - 1, total * t / T) -
                         wsum.begin());
    };
    std::vector<std::vector<int32_t>> part((size_t)T);
    auto work = [&](int64_t t) {
        std::vector<int32_t> &out = part[(size_t)t];
        int32_t cand[FC_MAX_VARS], sub[FC_MAX_VARS];
        const int64_t ra = first_row(t), rb = first_row(t + 1);
        for (int64_t a = ra; a < rb; ++a)
            for (int64_t b = a + 1; b < bend[(size_t)a]; ++b) {
                std::copy(prev.at(a), prev.at(a) + k1, cand);
                cand[k1] = prev.at(b)[k1 - 1];
                bool ok = true;
                for (int32_t x = 0; ok && x < k - 2; ++x) {
                    int32_t u = 0;
                    for (int32_t t2 = 0; t2 < k; ++t2)
                        if (t2 != x) sub[u++] = cand[t2];
                    ok = prev.find(sub) >= 0;
                }
                if (ok) out.insert(out.end(), cand, cand + k);
            }
    };
    if (T == 1) {
        work(0);
    } else {
        std::vector<std::thread> th;
        for (int64_t t = 0; t < T; ++t) th.emplace_back(work, t);
        for (auto &x : th) x.join();
    }
    std::vector<int32_t> all;
    size_t sz = 0;
    for (auto &p : part) sz += p.size();
    all.reserve(sz);
    for (auto &p : part) all.insert(all.end(), p.begin(), p.end());
    return all;
}

// Rule S - {X} => X of itemset i of level li (X = its item x): key is the
// antecedent's index in level li - 1, replaced by the antecedent's rank in
// tuple order once every level is known.
struct Rule {
    int64_t key;
    int32_t li, i, x;
    double conf;
};

// The rules of one level (itemsets of at least 2 items) against the level
// below, on host threads, in itemset order.  False when an antecedent is
// missing, which anti-monotonicity rules out for frequent itemsets.
bool level_rules(const Level &L, const Level &below, int32_t li, double minconf,
                 std::vector<Rule> &out) {
    const int64_t n = L.size();
    unsigned hw = std::thread::hardware_concurrency();
    const int64_t T = std::max<int64_t>(
        1, std::min<int64_t>((int64_t)std::min(16u, hw ? hw : 1u), n / 4096 + 1));
    std::vector<std::vector<Rule>> part((size_t)T);
    std::vector<char> bad((size_t)T, 0);
    auto work = [&](int64_t t) {
        int32_t ante[FC_MAX_VARS];
        for (int64_t i = n * t / T; i < n * (t + 1) / T; ++i) {
            const int32_t *sv = L.at(i);
            const int64_t cnt = L.count[(size_t)i];
            for (int32_t x = 0; x < L.k; ++x) {
                int32_t u = 0;
                for (int32_t t2 = 0; t2 < L.k; ++t2)
                    if (t2 != x) ante[u++] = sv[t2];
                const int64_t j = below.find(ante);
                if (j < 0) {
                    bad[(size_t)t] = 1;
                    return;
                }
                const double conf = (double)cnt / (double)below.count[(size_t)j];
                if (conf > minconf) part[(size_t)t].push_back({j, li, (int32_t)i, x, conf});
            }
        }
    };
    if (T == 1) {
        work(0);
    } else {
        std::vector<std::thread> th;
        for (int64_t t = 0; t < T; ++t) th.emplace_back(work, t);
        for (auto &x : th) x.join();
    }
    size_t sz = 0;
    for (int64_t t = 0; t < T; ++t) {
        if (bad[(size_t)t]) return false;
        sz += part[(size_t)t].size();
    }
    out.reserve(sz);
    for (auto &p : part) out.insert(out.end(), p.begin(), p.end());
    return true;
}

}  // namespace
}  // namespace fc

using namespace fc;

extern "C" int fc_mine(fc_db *db, const int32_t *items, int32_t ni, double minsup, double minconf,
                       int32_t max_size, fc_arm_result **out, void *stream) {
    clear_error();
    if (!db || !out || ni < 0 || (ni > 0 && !items) || max_size < 1) {
        set_error("fc_mine: need a database, items (ni >= 0), max_size >= 1 and out");
        return FC_ERR_INVALID;
    }
    if (max_size > FC_MAX_VARS) {
        set_error("fc_mine: itemsets of at most %d items (max_size = %d)", FC_MAX_VARS, max_size);
        return FC_ERR_INVALID;
    }
    *out = nullptr;
    std::vector<uint8_t> seen((size_t)db->n, 0);
    for (int32_t i = 0; i < ni; ++i) {
        const int32_t v = items[i];
        if (v < 0 || v >= db->n) {
            set_error("fc_mine: item %d out of range [0, %d)", v, db->n);
            return FC_ERR_INVALID;
        }
        if (db->arity[(size_t)v] != 2) {
            set_error("fc_mine: item %d is not binary (arity %d)", v, db->arity[(size_t)v]);
            return FC_ERR_INVALID;
        }
        if (seen[(size_t)v]++) {
            set_error("fc_mine: item %d appears twice", v);
            return FC_ERR_INVALID;
        }
    }
    auto *R = new (std::nothrow) fc_arm_result();
    if (!R) {
        set_error("fc_mine: host allocation failed");
        return FC_ERR_NOMEM;
    }
    struct Guard {
        fc_arm_result *r;
        ~Guard() { delete r; }
    } guard{R};
    const int64_t m = db->m;
    std::vector<Level> levels;
    levels.reserve((size_t)max_size);  // rule threads hold references into it
    // the rules of a level are generated on host threads while the device
    // counts the next level
    std::vector<std::vector<Rule>> lrules((size_t)max_size);
    std::vector<char> lok((size_t)max_size, 1);
    std::vector<std::thread> rtasks;
    struct Join {
        std::vector<std::thread> &t;
        ~Join() {
            for (auto &x : t)
                if (x.joinable()) x.join();
        }
    } join_rules{rtasks};
    auto start_rules = [&](int32_t li) {
        const Level *L = &levels[(size_t)li], *below = &levels[(size_t)li - 1];
        char *ok = &lok[(size_t)li];
        std::vector<Rule> *out = &lrules[(size_t)li];
        rtasks.emplace_back([=] { *ok = level_rules(*L, *below, li, minconf, *out) ? 1 : 0; });
    };

    // level 1: supports from the marginals (state 1 of each item)
    Level L1;
    L1.k = 1;
    {
        std::vector<int32_t> it(items, items + ni);
        std::sort(it.begin(), it.end());
        for (int32_t v : it) {
            const int64_t c = db->marg[(size_t)db->state_off[(size_t)v] + 1];
            if (frequent(c, m, minsup)) {
                L1.items.push_back(v);
                L1.count.push_back(c);
            }
        }
    }
    L1.index();  // subset lookups of the next level and of the rules
    levels.push_back(std::move(L1));

    // level 2: the Gram's pair records over the frequent items
    if (max_size >= 2 && levels[0].size() >= 2) {
        const Level &p = levels[0];
        const int32_t n1 = (int32_t)p.size();
        const int64_t cap = (int64_t)n1 * (n1 - 1) / 2;
        std::vector<fc_pair_rec> rec((size_t)std::max<int64_t>(cap, 1));
        int64_t n_out = 0;
        const int rc = fc_pairs(db, p.items.data(), n1, minsup, nullptr, rec.data(), cap, &n_out,
                                stream);
        if (rc != FC_OK) return rc;
        Level L2;
        L2.k = 2;
        for (int64_t r = 0; r < std::min(n_out, cap); ++r) {  // ordered by (a, b), a < b
            L2.items.push_back(p.items[(size_t)rec[(size_t)r].a]);
            L2.items.push_back(p.items[(size_t)rec[(size_t)r].b]);
            L2.count.push_back(rec[(size_t)r].n_ab);
        }
        L2.index();  // subset lookups of the next level and of the rules
        levels.push_back(std::move(L2));
        start_rules(1);
    }

    // levels 3..max_size: join, prune, count in batches, keep the frequent
    constexpr int64_t kBatch = int64_t(1) << 20;
    while ((int32_t)levels.size() >= 2 && (int32_t)levels.size() < max_size &&
           levels.back().size() >= 2) {
        const Level &prev = levels.back();
        const int32_t k = prev.k + 1;
        const std::vector<int32_t> cand = candidates(prev);
        const int64_t nc = (int64_t)cand.size() / k;
        Level L;
        L.k = k;
        std::vector<int64_t> off, cnt;
        std::vector<uint8_t> ones;
        for (int64_t lo = 0; lo < nc; lo += kBatch) {
            const int64_t nb = std::min(kBatch, nc - lo);
            off.resize((size_t)nb + 1);
            for (int64_t i = 0; i <= nb; ++i) off[(size_t)i] = i * k;
            ones.assign((size_t)(nb * k), 1);
            cnt.assign((size_t)nb, 0);
            const int rc = fc_count_assignments(db, cand.data() + lo * k, off.data(), ones.data(),
                                                nb, cnt.data(), stream);
            if (rc != FC_OK) return rc;
            for (int64_t i = 0; i < nb; ++i)
                if (frequent(cnt[(size_t)i], m, minsup)) {
                    L.items.insert(L.items.end(), cand.begin() + (lo + i) * k,
                                   cand.begin() + (lo + i + 1) * k);
                    L.count.push_back(cnt[(size_t)i]);
                }
        }
        if (L.size() == 0) break;
        L.index();  // subset lookups of the next level and of the rules
        levels.push_back(std::move(L));
        start_rules((int32_t)levels.size() - 1);
    }

    // itemsets, level by level
    {
        size_t ns = 0, nsi = 0;
        for (const Level &L : levels) {
            ns += (size_t)L.size();
            nsi += (size_t)L.size() * (size_t)L.k;
        }
        R->set_items.reserve(nsi);
        R->set_off.reserve(ns + 1);
        R->set_count.reserve(ns);
    }
    for (const Level &L : levels) {
        for (int64_t i = 0; i < L.size(); ++i) {
            R->set_items.insert(R->set_items.end(), L.at(i), L.at(i) + L.k);
            R->set_off.push_back((int64_t)R->set_items.size());
            R->set_count.push_back(L.count[(size_t)i]);
        }
    }
    // Rank of every itemset in tuple order (a proper prefix first): the
    // pre-order of the trie whose children of a (k-1)-itemset are the
    // k-itemsets extending it by one larger item -- a contiguous run of level
    // k, found by one merge of two sorted levels.
    const int32_t nl = (int32_t)levels.size();
    std::vector<std::vector<int64_t>> child0((size_t)nl), rank((size_t)nl);
    for (int32_t li = 0; li < nl; ++li) {
        const int64_t n = levels[(size_t)li].size();
        rank[(size_t)li].assign((size_t)n, 0);
        child0[(size_t)li].assign((size_t)n + 1, 0);
        if (li + 1 < nl) {
            const Level &up = levels[(size_t)li + 1], &L = levels[(size_t)li];
            int64_t c = 0;
            for (int64_t p = 0; p < n; ++p) {
                child0[(size_t)li][(size_t)p] = c;
                while (c < up.size() && std::equal(up.at(c), up.at(c) + L.k, L.at(p))) ++c;
            }
            child0[(size_t)li][(size_t)n] = c;
        }
    }
    {
        int64_t next = 0;
        std::vector<std::pair<int32_t, int64_t>> stack;  // (level, index)
        for (int64_t i = levels[0].size() - 1; i >= 0; --i) stack.push_back({0, i});
        while (!stack.empty()) {
            const auto [li, i] = stack.back();
            stack.pop_back();
            rank[(size_t)li][(size_t)i] = next++;
            if (li + 1 < nl)
                for (int64_t c = child0[(size_t)li][(size_t)i + 1] - 1;
                     c >= child0[(size_t)li][(size_t)i]; --c)
                    stack.push_back({li + 1, c});
        }
    }
    // rules S - {X} => X of every frequent S with |S| >= 2, level by level,
    // each keyed by its antecedent's rank
    for (auto &x : rtasks) x.join();
    std::vector<Rule> rules;
    {
        size_t nrl = 0;
        for (int32_t li = 1; li < nl; ++li) {
            if (!lok[(size_t)li]) {
                set_error("fc_mine: a subset of a frequent itemset is missing");
                return FC_ERR_DEVICE;
            }
            nrl += lrules[(size_t)li].size();
        }
        rules.reserve(nrl);
        for (int32_t li = 1; li < nl; ++li)
            for (Rule r : lrules[(size_t)li]) {
                r.key = rank[(size_t)li - 1][(size_t)r.key];
                rules.push_back(r);
            }
    }
    // order: counting sort by antecedent rank, then by consequent within one
    // antecedent (a handful of rules each)
    int64_t nsets = 0;
    for (const Level &L : levels) nsets += L.size();
    std::vector<int64_t> start((size_t)nsets + 1, 0);
    for (const Rule &r : rules) ++start[(size_t)r.key + 1];
    for (int64_t i = 0; i < nsets; ++i) start[(size_t)i + 1] += start[(size_t)i];
    std::vector<int64_t> ord(rules.size()), fill(start.begin(), start.end() - 1);
    for (int64_t q = 0; q < (int64_t)rules.size(); ++q)
        ord[(size_t)fill[(size_t)rules[(size_t)q].key]++] = q;
    auto cons_of = [&](int64_t q) {
        const Rule &r = rules[(size_t)q];
        return levels[(size_t)r.li].at(r.i)[r.x];
    };
    for (int64_t g = 0; g < nsets; ++g)
        if (start[(size_t)g + 1] - start[(size_t)g] > 1)
            std::sort(ord.begin() + start[(size_t)g], ord.begin() + start[(size_t)g + 1],
                      [&](int64_t a, int64_t b) { return cons_of(a) < cons_of(b); });
    const int64_t nr = (int64_t)rules.size();
    {
        size_t nri = 0;
        for (const Rule &r : rules) nri += (size_t)levels[(size_t)r.li].k - 1;
        R->rule_items.reserve(nri);
    }
    R->rule_cons.resize((size_t)nr);
    R->rule_support.resize((size_t)nr);
    R->rule_conf.resize((size_t)nr);
    R->rule_off.resize((size_t)nr + 1);
    R->rule_off[0] = 0;
    for (int64_t q = 0; q < nr; ++q) {
        const Rule &r = rules[(size_t)ord[(size_t)q]];
        const Level &L = levels[(size_t)r.li];
        const int32_t *sv = L.at(r.i);
        for (int32_t t = 0; t < L.k; ++t)
            if (t != r.x) R->rule_items.push_back(sv[t]);
        R->rule_off[(size_t)q + 1] = (int64_t)R->rule_items.size();
        R->rule_cons[(size_t)q] = sv[r.x];
        R->rule_support[(size_t)q] = (double)L.count[(size_t)r.i] / (double)m;
        R->rule_conf[(size_t)q] = r.conf;
    }
    *out = R;
    guard.r = nullptr;
    return FC_OK;
}

extern "C" int fc_arm_sizes(const fc_arm_result *r, int64_t *n_sets, int64_t *n_set_items,
                            int64_t *n_rules, int64_t *n_rule_items) {
    clear_error();
    if (!r || !n_sets || !n_set_items || !n_rules || !n_rule_items) {
        set_error("fc_arm_sizes: need a result and four outputs");
        return FC_ERR_INVALID;
    }
    *n_sets = (int64_t)r->set_count.size();
    *n_set_items = (int64_t)r->set_items.size();
    *n_rules = (int64_t)r->rule_cons.size();
    *n_rule_items = (int64_t)r->rule_items.size();
    return FC_OK;
}

extern "C" int fc_arm_read(const fc_arm_result *r, int32_t *set_items, int64_t *set_off,
                           int64_t *set_count, int32_t *rule_items, int64_t *rule_off,
                           int32_t *rule_cons, double *rule_support, double *rule_conf) {
    clear_error();
    if (!r) {
        set_error("fc_arm_read: need a result");
        return FC_ERR_INVALID;
    }
    auto put = [](auto *dst, const auto &v) {
        if (dst && !v.empty()) std::memcpy(dst, v.data(), sizeof(v[0]) * v.size());
    };
    put(set_items, r->set_items);
    put(set_off, r->set_off);
    put(set_count, r->set_count);
    put(rule_items, r->rule_items);
    put(rule_off, r->rule_off);
    put(rule_cons, r->rule_cons);
    put(rule_support, r->rule_support);
    put(rule_conf, r->rule_conf);
    return FC_OK;
}

extern "C" void fc_arm_free(fc_arm_result *r) { delete r; }

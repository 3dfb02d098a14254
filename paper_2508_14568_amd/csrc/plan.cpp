// Plans: every step is a list of bootstraps whose inputs are ready.
//
// Main loop (Algorithm 1/4): the cells of anti-diagonal s = i + j depend
// only on diagonal s - 1 (Section 6.2), so step s holds every query's cells
// with i + j = s.  Equality (Section 4, Algorithm 3 with the eq9 table of
// Algorithm 4) is independent of the DP; as in Algorithm 4 it runs inside
// the loop, each stage one step ahead of the cells that read it.  The key of a cell and the
// difference update are folded into the bootstrap's job (see launch.h).
// With Algorithm 1's band (Section 3.2) only the pairs and cells with
// |i - j| <= band get bootstraps, neighbours outside it read as Enc(1), and
// the result is the diagonal path of differences.  Section 3.1's noise
// refresh adds a step after every refresh-th diagonal that bootstraps the
// differences it wrote through the identity table.
#include "plan.h"

#include <algorithm>
#include <map>
#include <set>

#include "context.h"

namespace lvs {

namespace {

constexpr size_t W = kCtWords;
constexpr uint64_t kOne = uint64_t(1) << kDeltaLog;   // Enc(1) body of a noise-free ciphertext

int nsym(int encoding) { return encoding == LVS_ENC_ASCII7 ? 2 : 1; }

Job blank_job() {
    Job j{};
    return j;
}

struct Builder {
    Plan& P;
    explicit Builder(Plan& p) : P(p) {}
    void step() { P.steps.push_back({P.jobs.size(), 0}); }
    void add(const Job& j) {
        P.jobs.push_back(j);
        P.steps.back().count++;
    }
};

bool both_encrypted(const QuerySpec& q) { return q.B != nullptr && q.eq9_in == nullptr; }

}  // namespace

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

size_t band_cells(size_t m, size_t n, long band) {
    if (band < 0) return m * n;
    size_t c = 0;
    for (size_t i = 1; i <= m; ++i) {
        const size_t lo = i > size_t(band) ? i - size_t(band) : 1;
        const size_t hi = std::min(n, i + size_t(band));
        if (hi >= lo) c += hi - lo + 1;
    }
    return c;
}

size_t diagonal_cells(const QuerySpec& q, size_t s) {
    if (!q.m || !q.n || s < 2 || s > q.m + q.n) return 0;
    size_t lo = (s > q.n + 1) ? s - q.n : 1;
    size_t hi = std::min(q.m, s - 1);
    if (q.band >= 0) {
        // |i - (s - i)| <= band  <=>  (s - band) / 2 <= i <= (s + band) / 2
        const size_t b = size_t(q.band);
        if (s > b) lo = std::max(lo, (s - b + 1) / 2);
        hi = std::min(hi, (s + b) / 2);
    }
    return hi >= lo ? hi - lo + 1 : 0;
}

size_t query_buffer_bytes(const QuerySpec& q) {
    size_t b = align256(sizeof(uint64_t) * (q.m + 1) * W);
    if (!q.h_last) b += align256(sizeof(uint64_t) * std::max<size_t>(q.n, 1) * W);   // row state
    if (both_encrypted(q)) {
        if (!q.eq9_out) b += align256(sizeof(uint64_t) * q.m * q.n * W);                     // eq9
        if (q.encoding == LVS_ENC_ASCII7 && !q.eq1_out) b += align256(sizeof(uint64_t) * q.m * q.n * W);   // eq1
    }
    return b;
}

size_t query_jobs(const QuerySpec& q) {
    const size_t cells = band_cells(q.m, q.n, q.band);
    size_t refresh = 0;
    if (q.refresh > 0)
        for (size_t s = q.refresh; s < q.m + q.n; s += q.refresh) refresh += 2 * diagonal_cells(q, s);
    if (!both_encrypted(q)) return cells + refresh;
    return cells * (q.encoding == LVS_ENC_ASCII7 ? 3 : 2) + refresh;
}

size_t plan_bytes(size_t njobs, size_t max_step) {
    max_step = std::min(max_step, kMaxStep);
    return align256(sizeof(Job) * std::max<size_t>(njobs, 1)) +
           align256(sizeof(uint64_t) * keyswitch_part_words(int(std::max<size_t>(max_step, 1))));
}

void assign_buffers(std::vector<QuerySpec>& qs, uint8_t*& ws) {
    for (auto& q : qs) {
        q.V = reinterpret_cast<uint64_t*>(ws);
        ws += align256(sizeof(uint64_t) * (q.m + 1) * W);
        if (!q.h_last) {
            q.H = reinterpret_cast<uint64_t*>(ws);
            ws += align256(sizeof(uint64_t) * std::max<size_t>(q.n, 1) * W);
        }
        if (both_encrypted(q)) {
            if (q.eq9_out) {
                q.eq9 = q.eq9_out;
            } else {
                q.eq9 = reinterpret_cast<uint64_t*>(ws);
                ws += align256(sizeof(uint64_t) * q.m * q.n * W);
            }
            if (q.encoding == LVS_ENC_ASCII7) {
                if (q.eq1_out) {
                    q.eq1 = q.eq1_out;
                } else {
                    q.eq1 = reinterpret_cast<uint64_t*>(ws);
                    ws += align256(sizeof(uint64_t) * q.m * q.n * W);
                }
            }
        }
    }
}

namespace {

// Equality jobs of cell (i, j) (1-based) of a query with both strings
// encrypted: stage 1 is eq1 = PBS(x1 - y1; LUT_eq) for ASCII, or eq9 =
// PBS(x - y; LUT_eq9) for DNA; stage 2 is eq9 = PBS(2 (x2 - y2) + (1 - eq1);
// LUT_eq9) (ASCII only).
Job equality_job(const QuerySpec& q, size_t i, size_t j, int stage) {
    const size_t ns = nsym(q.encoding);
    const size_t c = (i - 1) * q.n + (j - 1);
    Job J = blank_job();
    if (stage == 1) {
        J.src[0] = q.A + ((i - 1) * ns) * W;
        J.src[1] = q.B + ((j - 1) * ns) * W;
        J.coef[0] = 1;
        J.coef[1] = -1;
        if (q.encoding == LVS_ENC_ASCII7) {
            J.lut = LVS_LUT_EQ;
            J.dst[0] = q.eq1 + c * W;
        } else {
            J.lut = LVS_LUT_EQ9;
            J.dst[0] = q.eq9 + c * W;
        }
    } else {
        J.src[0] = q.A + ((i - 1) * 2 + 1) * W;
        J.src[1] = q.B + ((j - 1) * 2 + 1) * W;
        J.src[2] = q.eq1 + c * W;
        J.coef[0] = 2;
        J.coef[1] = -2;
        J.coef[2] = -1;
        J.delta = kOne;
        J.lut = LVS_LUT_EQ9;
        J.dst[0] = q.eq9 + c * W;
    }
    return J;
}

// Cells (i, s - i) of anti-diagonal s inside the query's band.
template <typename F>
void for_diagonal(const QuerySpec& q, size_t s, F&& f) {
    if (!q.m || !q.n || s < 2 || s > q.m + q.n) return;
    const size_t i_lo = (s > q.n + 1) ? s - q.n : 1;
    const size_t i_hi = std::min(q.m, s - 1);
    for (size_t i = i_lo; i <= i_hi; ++i)
        if (in_band(q, i, s - i)) f(i, s - i);
}

}  // namespace

void build_edit_distance_plan(const std::vector<QuerySpec>& qs, Plan& P, bool with_dp, size_t quantum, size_t cap,
                              std::vector<long>* step_diag) {
    Builder b(P);
    size_t smax = 0;
    bool any_ascii = false;
    for (const auto& q : qs)
        if (q.m && q.n) {
            smax = std::max(smax, q.m + q.n);
            any_ascii |= both_encrypted(q) && q.encoding == LVS_ENC_ASCII7;
        }
    if (!with_dp) {
        // equality alone: every pair in one step per stage
        for (int stage = 1; stage <= (any_ascii ? 2 : 1); ++stage) {
            b.step();
            for (const auto& q : qs) {
                if (!both_encrypted(q) || (stage == 2 && q.encoding != LVS_ENC_ASCII7)) continue;
                for (size_t s = 2; s <= q.m + q.n; ++s)
                    for_diagonal(q, s, [&](size_t i, size_t j) { b.add(equality_job(q, i, j, stage)); });
            }
        }
        return;
    }
    for (const auto& q : qs) {
        if (q.band < 0) {
            // an empty first string leaves h[0, 1..n] = Enc(1) as the result
            if (q.m == 0 && q.n) P.fills.push_back({q.h_last, q.n});
            continue;
        }
        // band path entries that no bootstrap writes keep the OneMatrix 1:
        // v[1,0], and every path cell outside the band (all of them when a
        // string is empty)
        if (q.m == 0 || q.n == 0) {
            if (q.m + q.n) P.fills.push_back({q.path, q.m + q.n});
            continue;
        }
        P.fills.push_back({q.path, 1});
        const size_t mn = std::min(q.m, q.n);
        for (size_t k = 2; k <= mn; ++k)
            if (!in_band(q, k, k - 1)) P.fills.push_back({q.path + (2 * k - 2) * W, 1});
        for (size_t j = q.m + 1; j <= q.n; ++j)
            if (!in_band(q, q.m, j)) P.fills.push_back({q.path + (2 * q.m + (j - q.m - 1)) * W, 1});
        for (size_t i = q.n + 1; i <= q.m; ++i)
            if (!in_band(q, i, q.n)) P.fills.push_back({q.path + (2 * q.n + (i - q.n - 1)) * W, 1});
    }
    // Step t bootstraps the cells of anti-diagonal t (t >= 2).  Equality has
    // no dependence on the DP (Algorithm 4 evaluates it inside the loop, but
    // any earlier step will do): each cell's last equality stage must run by
    // step t - 1 and, for ASCII, its first stage by step t - 2.  Those
    // deadlines are met exactly; then, when a device round holds `quantum`
    // bootstraps, the last partial round of a step is filled with equality
    // jobs of later diagonals, earliest deadline first (a last stage only
    // once its first stage ran in an earlier step), never past `cap`.
    struct Diag {
        std::vector<std::pair<size_t, std::pair<size_t, size_t>>> cells;   // (query, (i, j)) with equality
        size_t n1 = 0, n1_before = 0, n2 = 0;   // first stages placed (in earlier steps), last stages placed
    };
    std::vector<Diag> eqd(smax + 3);
    for (size_t k = 0; k < qs.size(); ++k) {
        const QuerySpec& q = qs[k];
        if (!both_encrypted(q)) continue;
        for (size_t s = 2; s <= q.m + q.n; ++s)
            for_diagonal(q, s, [&](size_t i, size_t j) { eqd[s].cells.push_back({k, {i, j}}); });
    }
    // ASCII and DNA queries may share a plan: a DNA cell has one stage (eq9,
    // deadline s - 1), an ASCII cell two; keep them in separate lists
    std::vector<Diag> eqd2(smax + 3);     // cells with a single stage (DNA)
    for (size_t s = 0; s < eqd.size(); ++s) {
        std::vector<std::pair<size_t, std::pair<size_t, size_t>>> two, one;
        for (const auto& c : eqd[s].cells) (qs[c.first].encoding == LVS_ENC_ASCII7 ? two : one).push_back(c);
        eqd[s].cells.swap(two);
        eqd2[s].cells.swap(one);
    }
    auto place1 = [&](Diag& d, size_t count) {   // first stages (ASCII eq1, DNA eq9)
        for (size_t e = 0; e < count && d.n1 < d.cells.size(); ++e, ++d.n1) {
            const auto& c = d.cells[d.n1];
            b.add(equality_job(qs[c.first], c.second.first, c.second.second, 1));
        }
    };
    auto place2 = [&](Diag& d, size_t count) {   // ASCII last stages whose first stage ran earlier
        for (size_t e = 0; e < count && d.n2 < d.n1_before; ++e, ++d.n2) {
            const auto& c = d.cells[d.n2];
            b.add(equality_job(qs[c.first], c.second.first, c.second.second, 2));
        }
    };
    const size_t all = size_t(-1);
    // fill the current step's last partial round, earliest deadline first
    // (the step precedes diagonal t + 1)
    auto fill = [&](size_t t) {
        if (quantum > 0) {
            const size_t count = P.steps.back().count;
            size_t target = (count + quantum - 1) / quantum * quantum;
            if (cap > 0) target = std::min(target, cap);
            for (size_t s = t + 2; s <= smax && P.steps.back().count < target; ++s) {
                // deadline s - 1: last stages of diagonal s, single stages of s
                place2(eqd[s], target - P.steps.back().count);
                place1(eqd2[s], target - P.steps.back().count);
                // deadline s - 1 as well: first stages of diagonal s + 1
                if (s + 1 <= smax) place1(eqd[s + 1], target - P.steps.back().count);
            }
        }
        for (auto& d : eqd) d.n1_before = d.n1;
    };
    const size_t t0 = any_ascii ? 0 : 1;
    for (size_t t = t0; t <= smax; ++t) {
        b.step();
        if (step_diag) step_diag->push_back(long(t));
        // deadlines: last stages of diagonal t + 1, first stages of diagonal t + 2
        if (t + 1 <= smax) {
            place2(eqd[t + 1], all);
            place1(eqd2[t + 1], all);
        }
        if (t + 2 <= smax) place1(eqd[t + 2], all);
        for (const auto& q : qs) {
            uint64_t* H = (q.h_last ? q.h_last : q.H) - W;   // H[j] = h[latest i, j], j >= 1
            for_diagonal(q, t, [&](size_t i, size_t j) {
                const uint64_t* eq;
                if (q.eq9_in) eq = q.eq9_in + ((i - 1) * q.n + (j - 1)) * W;
                else if (q.B) eq = q.eq9 + ((i - 1) * q.n + (j - 1)) * W;
                else eq = q.table + (size_t(q.cols[j - 1]) * q.m + (i - 1)) * W;
                // v_in = v[i, j-1] (Enc(1) on the left border and outside the
                // band), h_in = h[i-1, j] (Enc(1) on the top border and outside
                // the band); key = 4 - v_in + 3 h_in + eq9
                const uint64_t* v_in = (j == 1 || !in_band(q, i, j - 1)) ? nullptr : q.V + i * W;
                const uint64_t* h_in = (i == 1 || !in_band(q, i - 1, j)) ? nullptr : H + j * W;
                Job J = blank_job();
                J.src[0] = v_in;
                J.src[1] = h_in;
                J.src[2] = eq;
                J.coef[0] = -1;
                J.coef[1] = 3;
                J.coef[2] = 1;
                J.delta = 4 * kOne - (v_in ? 0 : kOne) + (h_in ? 0 : 3 * kOne);
                J.lut = LVS_LUT_MIN;
                // v[i,j] = M - h_in, h[i,j] = M - v_in
                J.dst[0] = q.V + i * W;
                J.sub[0] = h_in;
                J.sub_delta[0] = h_in ? 0 : kOne;
                J.dst[1] = H + j * W;
                J.sub[1] = v_in;
                J.sub_delta[1] = v_in ? 0 : kOne;
                J.dst[2] = q.trace ? q.trace + ((i - 1) * q.n + (j - 1)) * W : nullptr;
                if (q.band >= 0) {
                    // the band path: v[k,k-1] and h[k,k] for k <= min(m, n), then
                    // h[m, j > m] or v[i > n, n]
                    const size_t mn = std::min(q.m, q.n);
                    if (i == j) {
                        J.dst[3] = q.path + (2 * i - 1) * W;
                        J.copy_of = 1;
                    } else if (i == j + 1 && i <= mn) {
                        J.dst[3] = q.path + (2 * i - 2) * W;
                        J.copy_of = 0;
                    } else if (i == q.m && j > q.m) {
                        J.dst[3] = q.path + (2 * q.m + (j - q.m - 1)) * W;
                        J.copy_of = 1;
                    } else if (j == q.n && i > q.n) {
                        J.dst[3] = q.path + (2 * q.n + (i - q.n - 1)) * W;
                        J.copy_of = 0;
                    }
                }
                b.add(J);
            });
        }
        fill(t);
        // Section 3.1's refresh: the v and h just written on diagonal t are
        // bootstrapped in place through the identity table (the key switch
        // reads every source before the blind rotation writes)
        bool refresh = false;
        for (const auto& q : qs) refresh |= refresh_due(q, t) && diagonal_cells(q, t) > 0;
        if (!refresh) continue;
        b.step();
        if (step_diag) step_diag->push_back(-long(t) - 1);
        for (const auto& q : qs) {
            if (!refresh_due(q, t)) continue;
            uint64_t* H = (q.h_last ? q.h_last : q.H) - W;
            for_diagonal(q, t, [&](size_t i, size_t j) {
                for (uint64_t* x : {q.V + i * W, H + j * W}) {
                    Job J = blank_job();
                    J.src[0] = x;
                    J.coef[0] = 1;
                    J.lut = LVS_LUT_REFRESH;
                    J.dst[2] = x;
                    b.add(J);
                }
            });
        }
        fill(t);
    }
}

void build_preprocess_plan(const uint64_t* A, size_t m, int encoding, const std::vector<uint8_t>& syms_lo,
                           const std::vector<uint8_t>& syms_hi, uint64_t* table, uint64_t* eq1, Plan& P) {
    Builder b(P);
    const size_t alen = syms_lo.size();
    const size_t ns = nsym(encoding);
    // z1 = x1 - c1 (the cleartext symbol is a noise-free ciphertext)
    b.step();
    for (size_t c = 0; c < alen; ++c)
        for (size_t i = 0; i < m; ++i) {
            Job J = blank_job();
            J.src[0] = A + (i * ns) * W;
            J.coef[0] = 1;
            J.delta = uint64_t(0) - uint64_t(syms_lo[c]) * kOne;
            if (encoding == LVS_ENC_ASCII7) {
                J.lut = LVS_LUT_EQ;
                J.dst[0] = eq1 + (c * m + i) * W;
            } else {
                J.lut = LVS_LUT_EQ9;
                J.dst[0] = table + (c * m + i) * W;
            }
            b.add(J);
        }
    if (encoding != LVS_ENC_ASCII7) return;
    // z2 = 2 (x2 - c2) + (1 - eq1)
    b.step();
    for (size_t c = 0; c < alen; ++c)
        for (size_t i = 0; i < m; ++i) {
            Job J = blank_job();
            J.src[0] = A + (i * 2 + 1) * W;
            J.src[1] = eq1 + (c * m + i) * W;
            J.coef[0] = 2;
            J.coef[1] = -1;
            J.delta = kOne - 2 * uint64_t(syms_hi[c]) * kOne;
            J.lut = LVS_LUT_EQ9;
            J.dst[0] = table + (c * m + i) * W;
            b.add(J);
        }
}

void build_pbs_plan(const uint64_t* in, const uint8_t* lut_ids, int lut, size_t B, uint64_t* out, Plan& P) {
    Builder b(P);
    b.step();
    for (size_t k = 0; k < B; ++k) {
        Job J = blank_job();
        J.src[0] = in + k * W;
        J.coef[0] = 1;
        J.lut = uint32_t(lut_ids ? lut_ids[k] : lut);
        J.dst[2] = out + k * W;
        b.add(J);
    }
}

size_t wide_buffer_bytes(size_t pairs, size_t c) {
    if (c <= 1) return 0;
    return align256(sizeof(uint64_t) * pairs * c * W) + align256(sizeof(uint64_t) * pairs * ((c + 14) / 15) * W);
}

size_t wide_jobs(size_t pairs, size_t c) {
    size_t jobs = pairs * c;
    for (size_t cnt = c; cnt > 1;) {
        cnt = (cnt + 14) / 15;
        jobs += pairs * cnt;
    }
    return jobs;
}

size_t wide_max_step(size_t pairs, size_t c) { return pairs * c; }

void build_wide_equality(Plan& P, size_t pairs, size_t c, WideChunkInput (*chunk)(const void*, size_t, size_t),
                         const void* ctx, uint64_t* out, uint8_t*& ws) {
    constexpr size_t kGroup = 15;   // Algorithm 2: groups of at most t - 1 for a 16-value lookup
    Builder b(P);
    uint64_t* buf[2] = {nullptr, nullptr};
    if (c > 1) {
        buf[0] = reinterpret_cast<uint64_t*>(ws);
        ws += align256(sizeof(uint64_t) * pairs * c * W);
        buf[1] = reinterpret_cast<uint64_t*>(ws);
        ws += align256(sizeof(uint64_t) * pairs * ((c + kGroup - 1) / kGroup) * W);
    }
    // sub-equality of every chunk pair: PBS(x_k - y_k; LUT_eq), or LUT_eq9
    // when one chunk is the whole symbol
    b.step();
    for (size_t p = 0; p < pairs; ++p)
        for (size_t k = 0; k < c; ++k) {
            const WideChunkInput in = chunk(ctx, p, k);
            Job J = blank_job();
            J.src[0] = in.a;
            J.coef[0] = 1;
            if (in.b) {
                J.src[1] = in.b;
                J.coef[1] = -1;
            } else {
                J.delta = uint64_t(0) - uint64_t(in.clear) * kOne;
            }
            J.lut = c == 1 ? LVS_LUT_EQ9 : LVS_LUT_EQ;
            J.dst[2] = c == 1 ? out + p * W : buf[0] + (p * c + k) * W;
            b.add(J);
        }
    // merging: groups of at most 15 summed, a group of g offset by 15 - g, so
    // that the sum reads 15 exactly when all g are 1; bootstrapped in place
    int cur = 0;
    for (size_t cnt = c; cnt > 1;) {
        const size_t G = (cnt + kGroup - 1) / kGroup;
        uint64_t* sums = buf[cur ^ 1];
        P.sums.push_back({buf[cur], sums, pairs, int(cnt), int(G), int(kGroup)});
        P.steps.push_back({P.jobs.size(), 0, int(P.sums.size() - 1)});
        b.step();
        for (size_t p = 0; p < pairs; ++p)
            for (size_t g = 0; g < G; ++g) {
                const size_t size = std::min(cnt, (g + 1) * kGroup) - g * kGroup;
                Job J = blank_job();
                J.src[0] = sums + (p * G + g) * W;
                J.coef[0] = 1;
                J.delta = uint64_t(kGroup - size) * kOne;
                J.lut = G == 1 ? LVS_LUT_MAX9 : LVS_LUT_MAX;
                J.dst[2] = G == 1 ? out + p * W : sums + (p * G + g) * W;
                b.add(J);
            }
        cnt = G;
        cur ^= 1;
    }
}

size_t wide_levels(size_t c) {
    size_t L = 0;
    for (size_t cnt = c; cnt > 1; cnt = (cnt + 14) / 15) ++L;
    return L;
}

size_t wide_interleaved_bytes(size_t pairs, size_t c) {
    if (c <= 1) return 0;
    size_t b = align256(sizeof(uint64_t) * pairs * c * W);
    for (size_t cnt = c; cnt > 1;) {
        cnt = (cnt + 14) / 15;
        b += align256(sizeof(uint64_t) * pairs * cnt * W);
    }
    return b;
}

size_t wide_step_bound(const std::vector<QuerySpec>& qs, size_t c) {
    size_t per = 1 + c;   // a cell, its chunk sub-equalities and its merges
    for (size_t cnt = c; cnt > 1;) {
        cnt = (cnt + 14) / 15;
        per += cnt;
    }
    size_t width = 0;
    for (const auto& q : qs) width += std::min(q.m, q.n);
    return width * per + 1024;
}

void build_wide_edit_distance_plan(const std::vector<QuerySpec>& qs, const std::vector<WideQuery>& wq, size_t c,
                                   size_t quantum, size_t cap, uint8_t*& ws, Plan& P) {
    constexpr size_t kGroup = 15;   // Algorithm 2: groups of at most t - 1 for a 16-value lookup
    // the main loop alone: one step per anti-diagonal t = 1 .. smax, each
    // followed by a refresh step when one is due
    Plan Pd;
    std::vector<long> step_diag;
    build_edit_distance_plan(qs, Pd, true, 0, 0, &step_diag);
    size_t smax = 0;
    for (const auto& q : qs)
        if (q.m && q.n) smax = std::max(smax, q.m + q.n);
    std::vector<size_t> dp_step(smax + 1, size_t(-1)), refresh_step(smax + 1, size_t(-1));
    for (size_t k = 0; k < step_diag.size(); ++k) {
        const long d = step_diag[k];
        if (d >= 0 && size_t(d) <= smax) dp_step[size_t(d)] = k;
        else if (d < 0 && size_t(-d - 1) <= smax) refresh_step[size_t(-d - 1)] = k;
    }
    // the pairs that need equality, in anti-diagonal order (so that the
    // pairs of one diagonal are one range of every level buffer)
    struct Pair {
        size_t k, i, j;
    };
    std::vector<Pair> pairs;
    std::vector<size_t> first(smax + 2, 0), count(smax + 2, 0);
    for (size_t s = 2; s <= smax; ++s) {
        first[s] = pairs.size();
        for (size_t k = 0; k < qs.size(); ++k)
            for_diagonal(qs[k], s, [&](size_t i, size_t j) { pairs.push_back({k, i, j}); });
        count[s] = pairs.size() - first[s];
    }
    const size_t D = pairs.size();
    // merging levels: level l sums groups of cnt[l - 1] into G[l] = cnt[l]
    const size_t L = wide_levels(c);
    std::vector<size_t> cnt(L + 1);
    cnt[0] = c;
    for (size_t l = 1; l <= L; ++l) cnt[l] = (cnt[l - 1] + kGroup - 1) / kGroup;
    std::vector<uint64_t*> buf(L + 1, nullptr);   // [D][cnt[l]]: chunk outputs (l = 0), level-l sums
    if (c > 1)
        for (size_t l = 0; l <= L; ++l) {
            buf[l] = reinterpret_cast<uint64_t*>(ws);
            ws += align256(sizeof(uint64_t) * D * cnt[l] * W);
        }
    auto eq9_of = [&](const Pair& x) {
        return wq[x.k].eq9 + ((x.i - 1) * qs[x.k].n + (x.j - 1)) * W;
    };
    // stage 0 of diagonal s: the chunk sub-equalities PBS(x_k - y_k; LUT_eq)
    // (LUT_eq9 into eq9 when one chunk is the whole symbol), placed in order
    std::vector<size_t> placed0(smax + 2, 0);
    Builder b(P);
    auto place0 = [&](size_t s, size_t n) {
        const size_t total = count[s] * c;
        for (size_t e = 0; e < n && placed0[s] < total; ++e, ++placed0[s]) {
            const size_t d = first[s] + placed0[s] / c, kk = placed0[s] % c;
            const Pair& x = pairs[d];
            Job J = blank_job();
            J.src[0] = wq[x.k].A + ((x.i - 1) * c + kk) * W;
            J.src[1] = wq[x.k].B + ((x.j - 1) * c + kk) * W;
            J.coef[0] = 1;
            J.coef[1] = -1;
            J.lut = c == 1 ? LVS_LUT_EQ9 : LVS_LUT_EQ;
            J.dst[2] = c == 1 ? eq9_of(x) : buf[0] + (d * c + kk) * W;
            b.add(J);
        }
    };
    // Slot t holds the cells of anti-diagonal t and, for diagonal s, stage 0
    // at slot s - (L + 1) and merging level l at slot s - (L + 1) + l (its
    // group sums as a linear step just before), so every eq9 of diagonal s is
    // written at slot s - 1.  Stage 0 may run earlier: the last partial
    // device round of a slot is filled with stage-0 jobs of later diagonals,
    // earliest first.
    const long S = long(L) + 1;
    for (long t = 2 - S; t <= long(smax); ++t) {
        for (size_t l = 1; l <= L; ++l) {
            const long s = t + S - long(l);
            if (s < 2 || s > long(smax) || count[size_t(s)] == 0) continue;
            const size_t f = first[size_t(s)];
            P.sums.push_back({buf[l - 1] + f * cnt[l - 1] * W, buf[l] + f * cnt[l] * W, count[size_t(s)],
                              int(cnt[l - 1]), int(cnt[l]), int(kGroup)});
            P.steps.push_back({P.jobs.size(), 0, int(P.sums.size() - 1)});
        }
        b.step();
        if (t >= 0 && dp_step[size_t(t)] != size_t(-1)) {
            const PlanStep& st = Pd.steps[dp_step[size_t(t)]];
            for (size_t x = st.off; x < st.off + st.count; ++x) b.add(Pd.jobs[x]);
        }
        for (size_t l = 1; l <= L; ++l) {
            const long s = t + S - long(l);
            if (s < 2 || s > long(smax)) continue;
            for (size_t d = first[size_t(s)]; d < first[size_t(s)] + count[size_t(s)]; ++d)
                for (size_t g = 0; g < cnt[l]; ++g) {
                    const size_t size = std::min(cnt[l - 1], (g + 1) * kGroup) - g * kGroup;
                    uint64_t* sum = buf[l] + (d * cnt[l] + g) * W;
                    Job J = blank_job();
                    J.src[0] = sum;
                    J.coef[0] = 1;
                    J.delta = uint64_t(kGroup - size) * kOne;
                    J.lut = cnt[l] == 1 ? LVS_LUT_MAX9 : LVS_LUT_MAX;
                    J.dst[2] = cnt[l] == 1 ? eq9_of(pairs[d]) : sum;
                    b.add(J);
                }
        }
        const long s0 = t + S;
        if (s0 >= 2 && s0 <= long(smax)) place0(size_t(s0), size_t(-1));
        if (quantum > 0) {
            size_t target = (P.steps.back().count + quantum - 1) / quantum * quantum;
            if (cap > 0) target = std::min(target, cap);
            for (long s = std::max<long>(s0 + 1, 2); s <= long(smax) && P.steps.back().count < target; ++s)
                place0(size_t(s), target - P.steps.back().count);
        }
        if (t >= 0 && refresh_step[size_t(t)] != size_t(-1)) {
            b.step();
            const PlanStep& st = Pd.steps[refresh_step[size_t(t)]];
            for (size_t x = st.off; x < st.off + st.count; ++x) b.add(Pd.jobs[x]);
        }
    }
    P.fills.insert(P.fills.end(), Pd.fills.begin(), Pd.fills.end());
}

size_t verify_plan(const Plan& P, size_t round, size_t cap, size_t* rounds) {
    // Sweeping the steps in order: a word that some job or group sum of the
    // plan writes may only be read (as a source or a subtrahend) once an
    // earlier step has written it.  Within a step the key switch reads the
    // sources' masks in a launch of its own, but the blind rotation reads
    // every source's body word and every subtrahend while other workgroups
    // of the same launch write their outputs, so a source or subtrahend that
    // another job of the same step writes, or a word two jobs of a step
    // write, is a race (a job may read what it writes itself: an in-place
    // refresh).  No step may exceed cap (0: no bound).
    auto sum_words = [](const SumOp& o, bool out, auto&& f) {
        const size_t per = size_t(out ? o.groups : o.cnt);
        const uint64_t* base = out ? o.out : o.in;
        for (size_t x = 0; x < o.items * per; ++x) f(uintptr_t(base + x * W));
    };
    std::set<uintptr_t> produced, seen;
    for (const Job& J : P.jobs)
        for (int d = 0; d < 4; ++d)
            if (J.dst[d]) produced.insert(uintptr_t(J.dst[d]));
    for (const SumOp& o : P.sums) sum_words(o, true, [&](uintptr_t a) { produced.insert(a); });
    size_t bad = 0, nrounds = 0;
    const size_t r = std::max<size_t>(round, 1);
    for (const PlanStep& S : P.steps) {
        if (S.sum >= 0) {
            const SumOp& o = P.sums[size_t(S.sum)];
            sum_words(o, false, [&](uintptr_t a) { bad += produced.count(a) && !seen.count(a); });
            sum_words(o, true, [&](uintptr_t a) { seen.insert(a); });
            continue;
        }
        nrounds += (S.count + r - 1) / r;
        if (cap && S.count > cap) ++bad;
        std::map<uintptr_t, size_t> writer;
        for (size_t x = S.off; x < S.off + S.count; ++x) {
            const Job& J = P.jobs[x];
            const void* reads[5] = {J.src[0], J.src[1], J.src[2], J.sub[0], J.sub[1]};
            for (const void* rd : reads)
                if (rd && produced.count(uintptr_t(rd)) && !seen.count(uintptr_t(rd))) ++bad;
            for (int d = 0; d < 4; ++d) {
                if (!J.dst[d]) continue;
                auto ins = writer.emplace(uintptr_t(J.dst[d]), x);
                if (!ins.second && ins.first->second != x) ++bad;
            }
        }
        for (size_t x = S.off; x < S.off + S.count; ++x) {
            const Job& J = P.jobs[x];
            const void* reads[5] = {J.src[0], J.src[1], J.src[2], J.sub[0], J.sub[1]};
            for (const void* rd : reads) {
                if (!rd) continue;
                auto it = writer.find(uintptr_t(rd));
                if (it != writer.end() && it->second != x) ++bad;
            }
        }
        for (const auto& w : writer) seen.insert(w.first);
    }
    if (rounds) *rounds = nrounds;
    return bad;
}

hipError_t upload_plan(Plan& P, uint8_t*& ws, hipStream_t st) {
    // split oversized steps (their jobs are independent); linear steps stay
    std::vector<PlanStep> steps;
    for (const auto& s : P.steps) {
        if (s.sum >= 0) {
            steps.push_back(s);
            continue;
        }
        for (size_t o = 0; o < s.count; o += kMaxStep) steps.push_back({s.off + o, std::min(kMaxStep, s.count - o)});
    }
    P.steps.swap(steps);
    P.max_step = 0;
    for (const auto& s : P.steps) P.max_step = std::max(P.max_step, s.count);
    P.d_jobs = reinterpret_cast<Job*>(ws);
    ws += align256(sizeof(Job) * std::max<size_t>(P.jobs.size(), 1));
    P.d_part = reinterpret_cast<uint64_t*>(ws);
    ws += align256(sizeof(uint64_t) * keyswitch_part_words(int(std::max<size_t>(P.max_step, 1))));
    if (P.jobs.empty()) return hipSuccess;
    hipError_t e = hipMemcpyAsync(P.d_jobs, P.jobs.data(), sizeof(Job) * P.jobs.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);     // the host copy may change after return
}

namespace {
hipError_t launch_steps(Context* C, const Plan& P, hipStream_t st, bool timed, size_t first = 0,
                        size_t count = SIZE_MAX, bool fills = true) {
    if (fills)
        for (const auto& f : P.fills) {
            hipError_t e = launch_trivial(f.first, int(f.second), 1, st);
            if (e != hipSuccess) return e;
        }
    const size_t last = std::min(P.steps.size(), count > P.steps.size() ? P.steps.size() : first + count);
    for (size_t x = first; x < last; ++x) {
        const PlanStep& s = P.steps[x];
        if (s.sum >= 0) {
            const SumOp& o = P.sums[size_t(s.sum)];
            hipError_t e = launch_group_sum(o.in, o.out, o.items, o.cnt, o.groups, o.group, C->cus, st);
            if (e != hipSuccess) return e;
            continue;
        }
        if (!s.count) continue;
        const int B = int(s.count);
        const int ns = keyswitch_splits(B, C->ks_tile);
        {
            TimedLaunch t(C, timed ? kProfKeySwitch : -1, uint64_t(B));
            hipError_t e = launch_keyswitch_jobs(P.d_jobs + s.off, B, C->ksk, P.d_part, st, ns, C->ks_tile);
            if (e != hipSuccess) return e;
        }
        {
            TimedLaunch t(C, timed ? br_profile_id(C, B) : -1, uint64_t(B));
            hipError_t e = launch_blind_rotate_jobs(P.d_jobs + s.off, B, P.d_part, C->luts, C->bsk, C->tables,
                                                    C->br_grid, C->latency_form_max, C->latency_waves, st, ns,
                                                    C->throughput_waves);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}
}  // namespace

hipError_t run_plan_steps(Context* C, const Plan& P, size_t first, size_t count) {
    if (first == 0)
        for (const auto& f : P.fills) {
            hipError_t e = launch_trivial(f.first, int(f.second), 1, C->stream);
            if (e != hipSuccess) return e;
        }
    return launch_steps(C, P, C->stream, true, first, count, false);
}

hipError_t run_plan(Context* C, const Plan& P) {
    if (P.graph) {
        TimedLaunch t(C, kProfGraph, uint64_t(P.pbs()));
        return hipGraphLaunch(P.graph, C->stream);
    }
    return launch_steps(C, P, C->stream, true);
}

hipError_t capture_plan(Context* C, Plan& P) {
    hipError_t e;
    if (!C->capture_stream) {
        e = hipStreamCreateWithFlags(&C->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    e = hipStreamBeginCapture(C->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const bool prof = C->profiling;
    C->profiling = false;   // no events inside the graph
    hipError_t le = launch_steps(C, P, C->capture_stream, false);
    C->profiling = prof;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(C->capture_stream, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);   // the capture's own error is the one to report
        return le;
    }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&P.graph, g, nullptr, nullptr, 0);
    const hipError_t d = hipGraphDestroy(g);   // the executable does not need the graph
    return e != hipSuccess ? e : d;
}

}  // namespace lvs

// Autotuner of the ingest launch parameters (workgroup size, LDS rows, gutter
// split threshold, persistent grid).  Candidates are timed with HIP events on a
// scratch graph of the same shape, so the caller's sketches are never touched.
#include <algorithm>
#include <vector>

#include "gz_internal.h"

using namespace gz;

namespace {

struct Cand {
    gz_tuning t;
    float ms;
};

std::vector<gz_tuning> candidates(uint32_t P, uint32_t B, bool wide) {
    // workgroup sizes with at least 85% of lanes busy (J = wg / P groups of P lanes)
    std::vector<std::pair<double, uint32_t>> wgs;
    for (uint32_t wg = 64; wg <= 1024; wg += 64) {
        if (wg < P) continue;
        const double use = (double)((wg / P) * P) / wg;
        if (use >= 0.85) wgs.push_back({use, wg});
    }
    if (wgs.empty()) wgs.push_back({0.0, std::min<uint32_t>(1024, (P + 63) / 64 * 64)});
    std::vector<uint32_t> wg_list;
    for (auto& w : wgs)
        if (w.second >= 128 || wgs.size() == 1) wg_list.push_back(w.second);
    if (wg_list.empty()) wg_list.push_back(wgs.front().second);
    if (wg_list.size() > 5) {
        // keep a spread: smallest, largest and three in between
        std::vector<uint32_t> keep;
        for (int k = 0; k < 5; ++k) keep.push_back(wg_list[k * (wg_list.size() - 1) / 4]);
        keep.erase(std::unique(keep.begin(), keep.end()), keep.end());
        wg_list = keep;
    }
    std::vector<uint32_t> rows = {B, std::min<uint32_t>(B, 16u), std::min<uint32_t>(B, 12u)};
    std::sort(rows.begin(), rows.end());
    rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
    const uint32_t chunks[] = {4096u, 16384u, 65536u};
    std::vector<gz_tuning> out;
    for (uint32_t wg : wg_list)
        for (uint32_t dl : rows) {
            const uint32_t smem = (uint32_t)update_smem_bytes(dl, B, P, wide);
            if (smem > 160 * 1024) continue;
            const uint32_t by_lds = std::max<uint32_t>(1, (160 * 1024) / smem);
            const uint32_t by_threads = std::max<uint32_t>(1, 2048 / wg);
            const uint32_t wmax = std::min<uint32_t>(8, std::min(by_lds, by_threads));
            std::vector<uint32_t> wpc = {wmax};
            if (wmax > 1) wpc.push_back((wmax + 1) / 2);
            for (uint32_t c : chunks)
                for (uint32_t w : wpc) out.push_back(gz_tuning{wg, dl, c, w, 0});
        }
    return out;
}

}  // namespace

extern "C" gz_status gz_autotune(gz_graph* g, const uint32_t* src, const uint32_t* dst, uint64_t N,
                                 uint32_t flags, hipStream_t stream, gz_tuning* best,
                                 float* best_ms) {
    if (!g || !src || !dst || N == 0) return fail(GZ_EINVAL, "null argument or empty sample");
    if (!(flags & GZ_DEVICE_PTR)) return fail(GZ_EINVAL, "the sample must be in device memory");
    gz_config cfg{};
    cfg.rounds = g->R;
    gz_graph* t = nullptr;
    gz_status st = gz_sketch_init(&t, g->V, g->seed, &cfg);
    if (st) return st;
    st = gz_profile_enable(t, 1);
    std::vector<Cand> res;
    if (!st) {
        for (const gz_tuning& c : candidates(g->P, g->B, g->wide)) {
            if (gz_set_tuning(t, &c) != GZ_OK) continue;
            float bestc = 1e30f;
            for (int rep = 0; rep < 2 && !st; ++rep) {
                gz_profile pr{};
                st = gz_ingest(t, src, dst, nullptr, N, GZ_DEVICE_PTR | GZ_ASYNC, stream);
                if (!st) st = gz_profile_last(t, &pr);
                if (!st) bestc = std::min(bestc, pr.ingest_ms);
            }
            if (st) break;
            res.push_back({c, bestc});
        }
    }
    gz_status fst = gz_flush(t);
    gz_free(t);
    if (st) return st;
    if (fst) return fst;
    if (res.empty()) return fail(GZ_ESTATE, "no candidate configuration could run");
    const Cand* w = &res[0];
    for (const Cand& c : res)
        if (c.ms < w->ms) w = &c;
    // second stage: the grouping block count, with the best kernel parameters fixed
    Cand bestc = *w;
    if (!st) {
        st = gz_sketch_init(&t, g->V, g->seed, &cfg);
        if (!st) st = gz_profile_enable(t, 1);
        const uint32_t gb_list[] = {32u, 64u, 128u, 256u, 512u};
        for (uint32_t gb : gb_list) {
            if (st) break;
            gz_tuning c = w->t;
            c.group_blocks = gb;
            if (gz_set_tuning(t, &c) != GZ_OK) continue;
            float bc = 1e30f;
            for (int rep = 0; rep < 2 && !st; ++rep) {
                gz_profile pr{};
                st = gz_ingest(t, src, dst, nullptr, N, GZ_DEVICE_PTR | GZ_ASYNC, stream);
                if (!st) st = gz_profile_last(t, &pr);
                if (!st) bc = std::min(bc, pr.ingest_ms);
            }
            if (!st && bc < bestc.ms) bestc = Cand{c, bc};
        }
        if (t) {
            gz_status f2 = gz_flush(t);
            gz_free(t);
            if (!st) st = f2;
        }
        if (st) return st;
    }
    w = &bestc;
    g->tuning = w->t;
    if (best) *best = w->t;
    if (best_ms) *best_ms = w->ms;
    return GZ_OK;
}

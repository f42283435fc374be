// Timing-based variant selection: the project's stand-in for the paper's
// self-adaptive kernel selection (Sec. 4.4), which times the balanced and the
// shared-memory static kernel on the current data and keeps the faster.  Here
// every forward candidate (static, wave per tile dispatched statically,
// pixel-wise 8x8 raster / cost-ordered, wave per 16x16 tile, wave per 32x32
// block, hybrid, Gaussian-wise) and every backward candidate (static, wave
// per tile dispatched statically, balanced 8x8 raster / cost-ordered, wave
// per 16x16 tile, wave per 32x32 block) is run on the caller's frame and
// timed with HIP events; the winners
// are returned and cached in a
// text file keyed by a workload signature (image size and log2 buckets of the
// pair count and of the 50th / 99th / 100th percentile tile-list lengths), so
// a later call on a similar workload skips the timing.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "common.h"

namespace bgs {

static std::mutex g_tune_mu;

static int log2_bucket(uint64_t v) {
    int b = 0;
    while (v > 1) {
        v >>= 1;
        ++b;
    }
    return b;
}

static bgs_status workload_key(const bgs_frame* f, hipStream_t stream, std::string& key) {
    const int TX = (f->width + TILE - 1) / TILE, TY = (f->height + TILE - 1) / TILE;
    const int nt = TX * TY;
    std::vector<uint32_t> rg(2 * (size_t)nt);
    BGS_HIP(hipMemcpyAsync(rg.data(), f->ranges, rg.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    BGS_HIP(hipStreamSynchronize(stream));
    std::vector<uint32_t> len(nt);
    uint64_t M = 0;
    for (int t = 0; t < nt; ++t) {
        len[t] = rg[2 * t + 1] - rg[2 * t];
        M += len[t];
    }
    std::sort(len.begin(), len.end());
    auto q = [&](double p) { return len.empty() ? 0u : len[(size_t)std::min<double>(nt - 1, p * (nt - 1))]; };
    std::ostringstream os;
    os << f->width << "x" << f->height << ":m" << log2_bucket(M) << ":p50_" << log2_bucket(q(0.5)) << ":p99_"
       << log2_bucket(q(0.99)) << ":max" << log2_bucket(q(1.0));
    key = os.str();
    return BGS_OK;
}

struct TuneEntry {
    std::string key;
    int fv, fs, fo, bv, bs, bo;
    float fms, bms;
};

static bool cache_lookup(const char* path, const std::string& key, TuneEntry& e) {
    if (!path || !*path) return false;
    std::ifstream in(path);
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        std::istringstream is(line);
        TuneEntry t;
        if (!(is >> t.key >> t.fv >> t.fs >> t.fo >> t.bv >> t.bs >> t.bo >> t.fms >> t.bms)) continue;
        if (t.key == key) {
            e = t;  // the last entry for a key wins
            found = true;
        }
    }
    return found;
}

static void cache_store(const char* path, const TuneEntry& e) {
    if (!path || !*path) return;
    std::ofstream out(path, std::ios::app);
    out << e.key << " " << e.fv << " " << e.fs << " " << e.fo << " " << e.bv << " " << e.bs << " " << e.bo << " "
        << e.fms << " " << e.bms << "\n";
}

}  // namespace bgs

using namespace bgs;

extern "C" bgs_status bgs_autotune(const bgs_frame* frame, const bgs_render_cfg* base, float* out_color,
                                   float* out_alpha, float* out_depth, float* final_T, int32_t* n_contrib,
                                   const float* dL_dcolor, float* dL_dmeans2D, float* dL_dconic_opacity,
                                   float* dL_drgb, void* ws, size_t ws_bytes, const char* cache_path,
                                   bgs_render_cfg* best_fwd, bgs_render_cfg* best_bwd, float* fwd_ms_out,
                                   float* bwd_ms_out, hipStream_t stream) {
    BGS_REQUIRE(frame && base && best_fwd && best_bwd, "bgs_autotune: null argument");
    std::lock_guard<std::mutex> lock(g_tune_mu);
    // candidates and results carry the base's background and order fields,
    // not its instrumentation outputs
    bgs_render_cfg plain = *base;
    plain.wg_trace = nullptr;
    plain.wg_trace_cap = 0;
    plain.n_examined = nullptr;
    base = &plain;
    std::string key;
    bgs_status st = workload_key(frame, stream, key);
    if (st != BGS_OK) return st;
    TuneEntry e;
    if (cache_lookup(cache_path, key, e)) {
        *best_fwd = *base;
        best_fwd->variant = e.fv;
        best_fwd->subtile = e.fs;
        best_fwd->order = e.fo & 15;  // flags ride in the order fields' upper bits
        best_fwd->flags = e.fo >> 4;
        *best_bwd = *base;
        best_bwd->variant = e.bv;
        best_bwd->subtile = e.bs;
        best_bwd->order = e.bo & 15;  // the backward's flags ride in the order field's upper bits
        best_bwd->flags = e.bo >> 4;
        if (fwd_ms_out) *fwd_ms_out = e.fms;
        if (bwd_ms_out) *bwd_ms_out = e.bms;
        return BGS_OK;
    }
    // variant, sub-tile, order, flags
    const int fwd_cands[][4] = {{BGS_STATIC, 16, BGS_ORDER_RASTER, 0},
                                {BGS_STATIC_WAVE, 16, BGS_ORDER_RASTER, 0},
                                {BGS_BALANCED_PIXEL, 8, BGS_ORDER_RASTER, 0},
                                {BGS_BALANCED_PIXEL, 8, BGS_ORDER_COST, 0},
                                {BGS_BALANCED_PIXEL, 16, BGS_ORDER_RASTER, 0},
                                {BGS_BALANCED_PIXEL, 16, BGS_ORDER_COST, 0},
                                {BGS_BALANCED_PIXEL, 16, BGS_ORDER_COST, BGS_FLAG_PERSISTENT},
                                {BGS_BALANCED_PIXEL, 32, BGS_ORDER_COST, 0},
                                {BGS_BALANCED_HYBRID, 8, BGS_ORDER_COST, 0},
                                {BGS_BALANCED_GAUSS, 8, BGS_ORDER_COST, 0}};
    const int bwd_cands[][4] = {{BGS_STATIC, 16, BGS_ORDER_RASTER, 0},
                                {BGS_STATIC_WAVE, 16, BGS_ORDER_RASTER, 0},
                                {BGS_BALANCED_PIXEL, 8, BGS_ORDER_RASTER, 0},
                                {BGS_BALANCED_PIXEL, 8, BGS_ORDER_COST, 0},
                                {BGS_BALANCED_PIXEL, 16, BGS_ORDER_RASTER, 0},
                                {BGS_BALANCED_PIXEL, 16, BGS_ORDER_COST, 0},
                                {BGS_BALANCED_PIXEL, 16, BGS_ORDER_COST, BGS_FLAG_PERSISTENT},
                                {BGS_BALANCED_PIXEL, 16, BGS_ORDER_COST, BGS_FLAG_SPLIT_WALKS},
                                {BGS_BALANCED_PIXEL, 32, BGS_ORDER_COST, 0}};
    hipEvent_t e0, e1;
    BGS_HIP(hipEventCreate(&e0));
    BGS_HIP(hipEventCreate(&e1));
    auto timed = [&](auto&& run, float& ms) -> bgs_status {
        bgs_status s = run();  // warm-up (and error check)
        if (s != BGS_OK) return s;
        BGS_HIP(hipEventRecord(e0, stream));
        for (int r = 0; r < 2; ++r) {
            s = run();
            if (s != BGS_OK) return s;
        }
        BGS_HIP(hipEventRecord(e1, stream));
        BGS_HIP(hipEventSynchronize(e1));
        BGS_HIP(hipEventElapsedTime(&ms, e0, e1));
        ms *= 0.5f;
        return BGS_OK;
    };
    float best_f = INFINITY, best_b = INFINITY;
    int bf = 0, bb = 0;
    for (int c = 0; c < (int)(sizeof(fwd_cands) / sizeof(fwd_cands[0])); ++c) {
        bgs_render_cfg cfg = *base;
        cfg.variant = fwd_cands[c][0];
        cfg.subtile = fwd_cands[c][1];
        cfg.order = fwd_cands[c][2];
        cfg.flags = fwd_cands[c][3];
        float ms = 0;
        st = timed([&] {
            return bgs_render_fwd(frame, &cfg, out_color, out_alpha, out_depth, final_T, n_contrib, ws, ws_bytes,
                                  stream);
        }, ms);
        if (st != BGS_OK) break;
        if (ms < best_f) {
            best_f = ms;
            bf = c;
        }
    }
    const int packed = base->flags & BGS_FLAG_PACKED_GRADS;  // backward candidates on gradient records
    if (st == BGS_OK && dL_dcolor && dL_dmeans2D && (packed || (dL_dconic_opacity && dL_drgb))) {
        // the backward walks the forward's n_contrib: render once with the winner
        bgs_render_cfg cfg = *base;
        cfg.variant = fwd_cands[bf][0];
        cfg.subtile = fwd_cands[bf][1];
        cfg.order = fwd_cands[bf][2];
        cfg.flags = fwd_cands[bf][3];
        st = bgs_render_fwd(frame, &cfg, out_color, out_alpha, out_depth, final_T, n_contrib, ws, ws_bytes, stream);
        for (int c = 0; st == BGS_OK && c < (int)(sizeof(bwd_cands) / sizeof(bwd_cands[0])); ++c) {
            bgs_render_cfg bc = *base;
            bc.variant = bwd_cands[c][0];
            bc.subtile = bwd_cands[c][1];
            bc.order = bwd_cands[c][2];
            bc.flags = bwd_cands[c][3] | packed;
            bc.split_color = out_color;  // the winner forward's outputs, rendered just above
            bc.split_depth = out_depth;
            float ms = 0;
            // gradients accumulate; their values are scratch here
            st = timed([&] {
                return bgs_render_bwd(frame, &bc, final_T, n_contrib, dL_dcolor, nullptr, nullptr, dL_dmeans2D,
                                      dL_dconic_opacity, dL_drgb, nullptr, ws, ws_bytes, stream);
            }, ms);
            if (st != BGS_OK) break;
            if (ms < best_b) {
                best_b = ms;
                bb = c;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != BGS_OK) return st;
    *best_fwd = *base;
    best_fwd->variant = fwd_cands[bf][0];
    best_fwd->subtile = fwd_cands[bf][1];
    best_fwd->order = fwd_cands[bf][2];
    best_fwd->flags = fwd_cands[bf][3];
    *best_bwd = *base;
    best_bwd->variant = bwd_cands[bb][0];
    best_bwd->subtile = bwd_cands[bb][1];
    best_bwd->order = bwd_cands[bb][2];
    best_bwd->flags = bwd_cands[bb][3] | packed;  // split walks: the caller sets split_color / split_depth
    if (fwd_ms_out) *fwd_ms_out = best_f;
    if (bwd_ms_out) *bwd_ms_out = std::isinf(best_b) ? -1.0f : best_b;
    TuneEntry ne{key, best_fwd->variant, best_fwd->subtile, best_fwd->order | (best_fwd->flags << 4),
                 best_bwd->variant, best_bwd->subtile, best_bwd->order | (best_bwd->flags << 4), best_f,
                 std::isinf(best_b) ? -1.0f : best_b};
    if (!std::isinf(best_b)) cache_store(cache_path, ne);
    return BGS_OK;
}

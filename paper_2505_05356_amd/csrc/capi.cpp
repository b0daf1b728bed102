// Host side of the C ABI declared in include/gftorf.h: argument validation,
// workspace carving and the launch sequences of the forward and backward
// passes.  Nothing here allocates device memory or synchronises, except
// gftorf_read_status.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "common.h"
#include "mlp.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* where) {
    return fail(GFTORF_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

bool tile_ok(int tw, int th) {
    return (tw == 8 && th == 8) || (tw == 16 && th == 16) || (tw == 32 && th == 8);
}


int build_params(int64_t n, int32_t F, const gftorf_config* c, gft::Params* P) {
    if (!c) return fail(GFTORF_EINVAL, "config is NULL");
    if (n < 0) return fail(GFTORF_EINVAL, "n < 0");
    if (F < 1) return fail(GFTORF_EINVAL, "n_frames must be >= 1");
    if (c->width < 1 || c->height < 1 || c->width > 32768 || c->height > 32768)
        return fail(GFTORF_EINVAL, "width/height out of range [1, 32768]");
    if (c->n_freq < 1 || c->n_freq > GFTORF_MAX_FREQ) return fail(GFTORF_EINVAL, "n_freq out of range");
    if (c->n_phase < 1 || c->n_phase > GFTORF_MAX_PHASE) return fail(GFTORF_EINVAL, "n_phase out of range");
    if (!tile_ok(c->tile_w, c->tile_h)) return fail(GFTORF_EINVAL, "tile shape must be 8x8, 16x16 or 32x8");
    if (!(c->alpha_max > 0.f && c->alpha_max < 1.f)) return fail(GFTORF_EINVAL, "alpha_max must be in (0, 1)");
    if (!(c->alpha_min >= 0.f && c->alpha_min < c->alpha_max)) return fail(GFTORF_EINVAL, "alpha_min must be in [0, alpha_max)");
    if (!(c->T_min >= 0.f && c->T_min < 1.f)) return fail(GFTORF_EINVAL, "T_min must be in [0, 1)");
    if (!std::isfinite(c->extent_sigma) || !(c->dilation >= 0.f) || !std::isfinite(c->dilation) ||
        !std::isfinite(c->near_z) || !std::isfinite(c->source_intensity))
        return fail(GFTORF_EINVAL, "non-finite option");
    if (c->bg_T_power != 1 && c->bg_T_power != 2) return fail(GFTORF_EINVAL, "bg_T_power must be 1 or 2");
    if (c->max_pairs < 0 || c->max_pairs > (int64_t)0xF0000000ll)
        return fail(GFTORF_EINVAL, "max_pairs out of range [0, 0xF0000000]");
    for (int i = 0; i < c->n_freq; ++i)
        if (!(c->freq_hz[i] > 0.0) || !std::isfinite(c->freq_hz[i])) return fail(GFTORF_EINVAL, "bad frequency");
    const int64_t M = n * (int64_t)F;
    if (M > (int64_t)0xFFFFFFFFll) return fail(GFTORF_EINVAL, "n * n_frames must be < 2^32");
    gft::Params& p = *P;
    std::memset(&p, 0, sizeof(p));
    p.n = n;
    p.F = F;
    p.W = c->width;
    p.H = c->height;
    p.tw = c->tile_w;
    p.th = c->tile_h;
    p.ntx = (c->width + c->tile_w - 1) / c->tile_w;
    p.nty = (c->height + c->tile_h - 1) / c->tile_h;
    p.n_tiles = p.ntx * p.nty;
    if ((int64_t)p.n_tiles * F > (int64_t)0x7FFFFFFF) return fail(GFTORF_EINVAL, "too many tiles");
    if (((p.ntx + 7) / 8) * ((p.nty + 7) / 8) > gft::kMaxGroupsPerFrame)
        return fail(GFTORF_EINVAL, "more than " + std::to_string(gft::kMaxGroupsPerFrame) +
                                       " groups of 8x8 tiles per frame; use a larger tile shape");
    p.nf = c->n_freq;
    p.nphi = c->n_phase;
    p.nq = p.nf * p.nphi;
    for (int i = 0; i < p.nf; ++i) p.freq[i] = c->freq_hz[i];
    for (int j = 0; j < p.nphi; ++j) {
        p.cphi[j] = (float)std::cos((double)c->phase[j]);
        p.sphi[j] = (float)std::sin((double)c->phase[j]);
    }
    p.alpha_min = c->alpha_min;
    p.alpha_max = c->alpha_max;
    p.T_min = c->T_min;
    p.extent = c->extent_sigma;
    p.dilation = c->dilation;
    p.near_z = c->near_z;
    p.s_int = c->source_intensity;
    p.bg_pow = c->bg_T_power;
    p.cap = (unsigned long long)c->max_pairs;
    return GFTORF_OK;
}

// Buffer holding the depth-sorted items after the forward.
int depth_buffer(const gft::Params& P) { return gft::depth_sort_passes(P.F) & 1; }

int check_gauss(const gftorf_gaussians* g) {
    if (!g) return fail(GFTORF_EINVAL, "gaussians is NULL");
    if (g->n > 0 && (!g->mean || !g->scale || !g->quat || !g->opacity_logit || (!g->rgb && !g->sh_rgb) ||
                     (!g->albedo && !g->sh_albedo)))
        return fail(GFTORF_EINVAL, "required Gaussian array is NULL (mean, scale, quat, opacity_logit, "
                                   "rgb or sh_rgb, albedo or sh_albedo)");
    if ((g->sh_rgb || g->sh_albedo) && (g->sh_degree < 0 || g->sh_degree > 3))
        return fail(GFTORF_EINVAL, "sh_degree must be in [0, 3]");
    return GFTORF_OK;
}

// ---- profiler ---------------------------------------------------------------
struct ProfRec {
    const char* name;
    int ev;   // index of the start event; stop = ev + 1
};
struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> events;
    std::vector<int> free_slots;      // start-event indices available
    std::vector<ProfRec> recs;
    std::map<std::string, std::pair<int64_t, double>> totals;
};
// One profiler per calling thread, like the error string: a thread times the
// launches it makes itself, and threads never share timing state.
thread_local Profiler g_prof;

}  // namespace

namespace gft {

int prof_start(const char* name, hipStream_t s) {
    if (!g_prof.on || g_prof.free_slots.empty()) return -1;
    const int ev = g_prof.free_slots.back();
    g_prof.free_slots.pop_back();
    if (hipEventRecord(g_prof.events[ev], s) != hipSuccess) {
        g_prof.free_slots.push_back(ev);
        return -1;
    }
    g_prof.recs.push_back({name, ev});
    return (int)g_prof.recs.size() - 1;
}

void prof_stop(int slot, hipStream_t s) {
    if (slot < 0) return;
    (void)hipEventRecord(g_prof.events[g_prof.recs[slot].ev + 1], s);
}

}  // namespace gft

extern "C" {

int gftorf_profile_begin(int32_t max_launches) {
    if (max_launches < 1) return fail(GFTORF_EINVAL, "max_launches must be >= 1");
    if (g_prof.on) return fail(GFTORF_EINVAL, "profiling already on");
    g_prof = Profiler();
    g_prof.events.resize(2 * (size_t)max_launches);
    for (auto& e : g_prof.events) {
        // device-scope release: the timestamps do not wait for a system-scope
        // cache write-back, which would inflate the measured kernel time
        hipError_t r = hipEventCreateWithFlags(&e, hipEventReleaseToDevice);
        if (r != hipSuccess) return hip_fail(r, "gftorf_profile_begin");
    }
    for (int i = max_launches - 1; i >= 0; --i) g_prof.free_slots.push_back(2 * i);
    g_prof.on = true;
    return GFTORF_OK;
}

int gftorf_profile_collect(void) {
    for (const ProfRec& r : g_prof.recs) {
        hipError_t e = hipEventSynchronize(g_prof.events[r.ev + 1]);
        if (e != hipSuccess) return hip_fail(e, "gftorf_profile_collect");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, g_prof.events[r.ev], g_prof.events[r.ev + 1]);
        if (e != hipSuccess) return hip_fail(e, "gftorf_profile_collect");
        auto& t = g_prof.totals[r.name];
        t.first += 1;
        t.second += ms;
        g_prof.free_slots.push_back(r.ev);
    }
    g_prof.recs.clear();
    return GFTORF_OK;
}

int gftorf_profile_end(gftorf_profile_entry* out, int32_t max_entries, int32_t* n_entries) {
    int rc = gftorf_profile_collect();
    g_prof.on = false;
    int n = 0;
    for (const auto& kv : g_prof.totals) {
        if (out && n < max_entries) {
            std::memset(&out[n], 0, sizeof(out[n]));
            std::strncpy(out[n].name, kv.first.c_str(), sizeof(out[n].name) - 1);
            out[n].launches = kv.second.first;
            out[n].total_ms = kv.second.second;
        }
        ++n;
    }
    if (n_entries) *n_entries = n;
    for (auto& e : g_prof.events) (void)hipEventDestroy(e);
    g_prof.events.clear();
    g_prof.free_slots.clear();
    return rc;
}


size_t gftorf_workspace_size(int64_t n, int32_t n_frames, const gftorf_config* cfg) {
    gft::Params P;
    if (build_params(n, n_frames, cfg, &P) != GFTORF_OK) return 0;
    return gft::carve(nullptr, n, n_frames, P.nf, P.ntx, P.nty, P.cap).bytes;
}

int gftorf_render_fwd(const gftorf_gaussians* g, const gftorf_frame* frames, int32_t n_frames,
                      const gftorf_config* cfg, const gftorf_outputs* out, void* ws,
                      size_t ws_bytes, void* stream) {
    int rc = check_gauss(g);
    if (rc) return rc;
    gft::Params P;
    if ((rc = build_params(g->n, n_frames, cfg, &P))) return rc;
    if (!frames) return fail(GFTORF_EINVAL, "frames is NULL");
    if (!out || !out->T_final || !out->n_contrib) return fail(GFTORF_EINVAL, "outputs: T_final and n_contrib are required");
    if (!ws) return fail(GFTORF_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(GFTORF_EINVAL, "workspace must be 256-byte aligned");
    const gft::Workspace w = gft::carve(ws, g->n, n_frames, P.nf, P.ntx, P.nty, P.cap);
    if (ws_bytes < w.bytes) return fail(GFTORF_ENOWS, "workspace too small: need " + std::to_string(w.bytes) + " bytes");
    hipStream_t s = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();

    // every Status field is written during the forward (no clearing launch)
    gft::launch_preprocess(P, *g, frames, w, s);
    const int dbuf = gft::launch_depth_sort(P, w, s);
    hipError_t e = gft::launch_binning(P, w, dbuf, s);
    if (e == hipSuccess) e = gft::launch_composite_fwd(P, frames, w, *out, s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "gftorf_render_fwd");
    return GFTORF_OK;
}

int gftorf_render_bwd(const gftorf_gaussians* g, const gftorf_frame* frames, int32_t n_frames,
                      const gftorf_config* cfg, const gftorf_outputs* saved, const float* d_rgb,
                      const float* d_quad, const float* d_depth, const gftorf_gaussians_grad* grad,
                      float* d_bg, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_gauss(g);
    if (rc) return rc;
    gft::Params P;
    if ((rc = build_params(g->n, n_frames, cfg, &P))) return rc;
    if (!frames) return fail(GFTORF_EINVAL, "frames is NULL");
    if (!saved || !saved->T_final || !saved->n_contrib) return fail(GFTORF_EINVAL, "saved: T_final and n_contrib are required");
    if (!grad) return fail(GFTORF_EINVAL, "grad is NULL");
    if (!ws) return fail(GFTORF_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(GFTORF_EINVAL, "workspace must be 256-byte aligned");
    const gft::Workspace w = gft::carve(ws, g->n, n_frames, P.nf, P.ntx, P.nty, P.cap);
    if (ws_bytes < w.bytes) return fail(GFTORF_ENOWS, "workspace too small: need " + std::to_string(w.bytes) + " bytes");
    hipStream_t s = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();

    gft::launch_fill_f32(w.grec, 0.f, (int64_t)gft::grad_floats(P.nf) * w.M, s);
    if (d_bg) gft::launch_fill_f32(d_bg, 0.f, (int64_t)n_frames * (3 + P.nq), s);
    hipError_t e = gft::launch_composite_bwd(P, frames, w, *saved, d_rgb, d_quad,
                                             d_depth, d_bg, s);
    if (e == hipSuccess) {
        gft::launch_preprocess_bwd(P, *g, frames, w, *grad, s);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return hip_fail(e, "gftorf_render_bwd");
    return GFTORF_OK;
}

int gftorf_read_status(const void* ws, gftorf_status* out, void* stream) {
    if (!ws || !out) return fail(GFTORF_EINVAL, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    gft::Status st;
    hipError_t e = hipMemcpyAsync(&st, ws, sizeof(st), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "gftorf_read_status");
    out->n_pairs = (int64_t)st.n_pairs;
    out->max_pairs = (int64_t)st.cap;
    out->overflow = (int32_t)st.overflow;
    out->nonfinite = (int32_t)st.nonfinite;
    out->overflow_seen = (int32_t)st.overflow_seen;
    out->sort_fault = st.magic == gft::kStatusMagic ? (int32_t)(st.sort_fault != 0u) : 0;
    out->n_pairs_seen = (int64_t)st.n_pairs_seen;
    out->n_evaluated = out->n_composited = 0;
    // the forward's per-work-item counts, summed here (the stream is idle)
    if (st.magic == gft::kStatusMagic && st.n_items > 0 && st.n_items <= (1ull << 26) &&
        st.wcount_off >= sizeof(gft::Status) && st.wcount_off % 8 == 0 && st.wcount_off < (1ull << 44)) {
        std::vector<uint2> wc((size_t)st.n_items);
        e = hipMemcpy(wc.data(), static_cast<const char*>(ws) + st.wcount_off, sizeof(uint2) * wc.size(),
                      hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "gftorf_read_status");
        unsigned long long ev = 0, co = 0;
        for (const uint2& c : wc) {
            ev += c.x;
            co += c.y;
        }
        out->n_evaluated = (int64_t)ev;
        out->n_composited = (int64_t)co;
    }
    if (st.overflow) return fail(GFTORF_EOVERFLOW, "pairs exceeded max_pairs: " + std::to_string(st.n_pairs));
    if (out->sort_fault) return fail(GFTORF_EHIP, "depth sort: a look-back wait gave up; the forward is invalid");
    return GFTORF_OK;
}

int gftorf_clear_status(void* ws, void* stream) {
    if (!ws) return fail(GFTORF_EINVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(GFTORF_EINVAL, "workspace must be 256-byte aligned");
    (void)hipGetLastError();
    gft::launch_fill_u32(static_cast<uint32_t*>(ws), 0u, (int64_t)(sizeof(gft::Status) / 4),
                         static_cast<hipStream_t>(stream));
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GFTORF_OK : hip_fail(e, "gftorf_clear_status");
}

int gftorf_copy_lists(const void* ws, int64_t n, int32_t n_frames, const gftorf_config* cfg,
                      uint32_t* pair_key, uint32_t* pair_item, int64_t pair_capacity,
                      uint32_t* depth_key, uint32_t* depth_item, uint32_t* item_count,
                      uint32_t* item_rect, uint32_t* tile_ranges, void* stream) {
    gft::Params P;
    int rc = build_params(n, n_frames, cfg, &P);
    if (rc) return rc;
    if (!ws) return fail(GFTORF_EINVAL, "workspace is NULL");
    const gft::Workspace w = gft::carve(const_cast<void*>(ws), n, n_frames, P.nf, P.ntx, P.nty, P.cap);
    hipStream_t s = static_cast<hipStream_t>(stream);
    gft::Status st;
    hipError_t e = hipMemcpyAsync(&st, ws, sizeof(st), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "gftorf_copy_lists");
    unsigned long long np = st.n_pairs < P.cap ? st.n_pairs : P.cap;
    if (pair_capacity >= 0 && np > (unsigned long long)pair_capacity) np = (unsigned long long)pair_capacity;
    const int db = depth_buffer(P);
    auto cp = [&](void* dst, const void* src, size_t bytes) {
        if (dst && bytes && e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
    };
    if (pair_key && np) {
        gft::launch_keys_from_ranges(P, w, pair_key, np, s);
        e = hipGetLastError();
    }
    cp(pair_item, w.tval, 4 * np);
    cp(depth_key, w.dkey[db], 4 * (size_t)w.M);
    cp(depth_item, w.dval[db], 4 * (size_t)w.M);
    cp(item_count, w.cnt, 4 * (size_t)w.M);
    if (item_rect && e == hipSuccess) {
        gft::launch_item_rects(w, db, reinterpret_cast<uint2*>(item_rect), s);
        e = hipGetLastError();
    }
    cp(tile_ranges, w.ranges, 8 * (size_t)P.F * P.n_tiles);
    if (e != hipSuccess) return hip_fail(e, "gftorf_copy_lists");
    return GFTORF_OK;
}

int gftorf_l2_loss_grad(const float* pred, const float* targets, const int32_t* frame_index,
                        int32_t n_frames, int64_t elems_per_frame, float weight, float* grad,
                        float* loss, void* stream) {
    if (!pred || !targets || !grad) return fail(GFTORF_EINVAL, "NULL argument");
    if (n_frames < 1 || elems_per_frame < 1) return fail(GFTORF_EINVAL, "empty loss");
    (void)hipGetLastError();
    gft::launch_l2_loss(pred, targets, frame_index, n_frames, elems_per_frame, weight, grad, loss,
                        static_cast<hipStream_t>(stream));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GFTORF_OK : hip_fail(e, "gftorf_l2_loss_grad");
}

int gftorf_adam_step(const gftorf_adam_group* groups, int32_t n_groups, int32_t* step, float beta1,
                     float beta2, float eps, void* stream) {
    if (!groups || n_groups < 1 || !step) return fail(GFTORF_EINVAL, "bad Adam arguments");
    for (int i = 0; i < n_groups; ++i)
        if (groups[i].n < 0 || (groups[i].n > 0 && (!groups[i].param || !groups[i].grad || !groups[i].m || !groups[i].v)))
            return fail(GFTORF_EINVAL, "bad Adam group " + std::to_string(i));
    for (int i = 0; i < n_groups; ++i)
        if (groups[i].decay_steps < 0 || groups[i].reserved != 0 ||
            (groups[i].decay_steps > 0 && !(groups[i].lr > 0.f && groups[i].lr_final > 0.f)))
            return fail(GFTORF_EINVAL, "bad learning-rate decay in Adam group " + std::to_string(i));
    (void)hipGetLastError();
    gft::launch_adam(groups, n_groups, step, beta1, beta2, eps, static_cast<hipStream_t>(stream));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GFTORF_OK : hip_fail(e, "gftorf_adam_step");
}

int gftorf_select_frames(gftorf_frame* frames, int32_t n_batch, const gftorf_frame* seq,
                         int32_t n_seq, const float* bg_table, int32_t n_bg, int32_t n_quad,
                         const int32_t* step, int32_t* frame_index, void* stream) {
    if (!frames || !seq || !step || n_batch < 1 || n_seq < 1) return fail(GFTORF_EINVAL, "bad frame selection arguments");
    if (bg_table && (n_bg < 1 || n_quad < 0 || n_quad > GFTORF_MAX_QUAD)) return fail(GFTORF_EINVAL, "bad background table");
    (void)hipGetLastError();
    gft::launch_select_frames(frames, n_batch, seq, n_seq, bg_table, n_bg, n_quad, step, frame_index,
                              static_cast<hipStream_t>(stream));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GFTORF_OK : hip_fail(e, "gftorf_select_frames");
}

// ---- deformation network -------------------------------------------------

namespace {
bool mlp_layout(const gftorf_mlp_config* cfg, int64_t n, int32_t n_times, bool training,
                gft::mlp::Layout* L) {
    return cfg && gft::mlp::make_layout(cfg->n_freq_x, cfg->n_freq_t, cfg->width, cfg->depth, n,
                                        n_times, training, L);
}

int mlp_call(const gftorf_mlp_config* cfg, const float* params, const float* x0, int64_t n,
             const float* times, const gftorf_frame* frames, int32_t n_times, void* ws,
             size_t ws_bytes, bool training, gft::mlp::Layout* L, gft::mlp::Call* c) {
    if (!mlp_layout(cfg, n, n_times, training, L))
        return fail(GFTORF_EINVAL, "unsupported network: width must be 256, depth 8, "
                                   "3 (1 + 2 L_x) + 1 + 2 L_t <= 96, 1 <= n_times <= 64");
    if (!params || !x0 || (!times && !frames) || !ws) return fail(GFTORF_EINVAL, "NULL pointer");
    if (!std::isfinite(cfg->pos_scale) || !std::isfinite(cfg->time_scale))
        return fail(GFTORF_EINVAL, "non-finite input scale");
    if (ws_bytes < L->bytes) return fail(GFTORF_ENOWS, "workspace too small for the network");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(GFTORF_EINVAL, "workspace must be 256-byte aligned");
    c->params = params;
    c->x0 = x0;
    c->sx = cfg->pos_scale;
    c->st = cfg->time_scale;
    for (int t = 0; t < gft::mlp::kMaxTimes; ++t) c->times[t] = (times && t < n_times) ? times[t] : 0.f;
    c->frames = times ? nullptr : frames;
    c->ws = static_cast<char*>(ws);
    return GFTORF_OK;
}
}  // namespace

int64_t gftorf_mlp_param_count(const gftorf_mlp_config* cfg) {
    gft::mlp::Layout L;
    return mlp_layout(cfg, 1, 1, false, &L) ? L.n_params : 0;
}

size_t gftorf_mlp_workspace_size(const gftorf_mlp_config* cfg, int64_t n, int32_t n_times,
                                 int32_t training) {
    gft::mlp::Layout L;
    return mlp_layout(cfg, n, n_times, training != 0, &L) ? L.bytes : 0;
}

int gftorf_mlp_fwd(const gftorf_mlp_config* cfg, const float* params, const float* x0, int64_t n,
                   const float* times, int32_t n_times, float* delta, int32_t save, void* ws,
                   size_t ws_bytes, void* stream) {
    gft::mlp::Layout L;
    gft::mlp::Call c;
    const int rc = mlp_call(cfg, params, x0, n, times, nullptr, n_times, ws, ws_bytes, save != 0, &L, &c);
    if (rc != GFTORF_OK) return rc;
    if (!delta) return fail(GFTORF_EINVAL, "NULL pointer");
    (void)hipGetLastError();
    const hipError_t e = gft::mlp::launch_fwd(L, c, delta, save != 0, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GFTORF_OK : hip_fail(e, "gftorf_mlp_fwd");
}

int gftorf_mlp_bwd(const gftorf_mlp_config* cfg, const float* params, const float* x0, int64_t n,
                   const float* times, int32_t n_times, const float* d_delta, float* d_params,
                   float* d_x0, void* ws, size_t ws_bytes, void* stream) {
    gft::mlp::Layout L;
    gft::mlp::Call c;
    const int rc = mlp_call(cfg, params, x0, n, times, nullptr, n_times, ws, ws_bytes, true, &L, &c);
    if (rc != GFTORF_OK) return rc;
    if (!d_delta || !d_params) return fail(GFTORF_EINVAL, "NULL pointer");
    (void)hipGetLastError();
    const hipError_t e = gft::mlp::launch_bwd(L, c, d_delta, d_params, d_x0, false, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GFTORF_OK : hip_fail(e, "gftorf_mlp_bwd");
}

namespace {
int mlp_decisions(const gftorf_mlp_config* cfg, int64_t n, int32_t n_times, uint8_t* dec, bool write,
                  void* ws, size_t ws_bytes, void* stream, const char* what) {
    gft::mlp::Layout L;
    if (!mlp_layout(cfg, n, n_times, true, &L))
        return fail(GFTORF_EINVAL, "unsupported network: width must be 256, depth 8, "
                                   "3 (1 + 2 L_x) + 1 + 2 L_t <= 96, 1 <= n_times <= 64");
    if (!dec || !ws) return fail(GFTORF_EINVAL, "NULL pointer");
    if (ws_bytes < L.bytes) return fail(GFTORF_ENOWS, "workspace too small for the training network");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(GFTORF_EINVAL, "workspace must be 256-byte aligned");
    (void)hipGetLastError();
    const hipError_t e = gft::mlp::launch_decisions(L, static_cast<char*>(ws), dec, write,
                                                    static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GFTORF_OK : hip_fail(e, what);
}
}  // namespace

int gftorf_mlp_get_decisions(const gftorf_mlp_config* cfg, int64_t n, int32_t n_times,
                             uint8_t* decisions, void* ws, size_t ws_bytes, void* stream) {
    return mlp_decisions(cfg, n, n_times, decisions, false, ws, ws_bytes, stream, "gftorf_mlp_get_decisions");
}

int gftorf_mlp_set_decisions(const gftorf_mlp_config* cfg, int64_t n, int32_t n_times,
                             const uint8_t* decisions, void* ws, size_t ws_bytes, void* stream) {
    return mlp_decisions(cfg, n, n_times, const_cast<uint8_t*>(decisions), true, ws, ws_bytes, stream,
                         "gftorf_mlp_set_decisions");
}

int gftorf_mlp_fwd_noalloc(const gftorf_mlp_config* cfg, const float* params, const float* x0,
                           int64_t n, const float* times, int32_t n_times, float* delta,
                           void* stream) {
    gft::mlp::Layout L;
    if (!mlp_layout(cfg, n, n_times, false, &L))
        return fail(GFTORF_EINVAL, "unsupported network: width must be 256, depth 8, "
                                   "3 (1 + 2 L_x) + 1 + 2 L_t <= 96, 1 <= n_times <= 64");
    if (L.bytes > gft::mlp::kNoAllocScratchBytes)
        return fail(GFTORF_ENOWS, "weight copies need " + std::to_string(L.bytes) +
                                      " bytes, more than the static scratch holds");
    if (!params || !x0 || !times || !delta) return fail(GFTORF_EINVAL, "NULL pointer");
    char* scratch = nullptr;
    hipError_t e = gft::mlp::noalloc_scratch(&scratch);
    if (e != hipSuccess) return hip_fail(e, "gftorf_mlp_fwd_noalloc (static scratch address)");
    gft::mlp::Call c;
    const int rc = mlp_call(cfg, params, x0, n, times, nullptr, n_times, scratch, L.bytes, false, &L, &c);
    if (rc != GFTORF_OK) return rc;
    (void)hipGetLastError();
    e = gft::mlp::launch_fwd(L, c, delta, false, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GFTORF_OK : hip_fail(e, "gftorf_mlp_fwd_noalloc");
}

int gftorf_mlp_fwd_frames(const gftorf_mlp_config* cfg, const float* params, const float* x0,
                          int64_t n, const gftorf_frame* frames, int32_t n_frames, float* delta,
                          int32_t save, void* ws, size_t ws_bytes, void* stream) {
    gft::mlp::Layout L;
    gft::mlp::Call c;
    if (!frames) return fail(GFTORF_EINVAL, "NULL pointer");
    const int rc = mlp_call(cfg, params, x0, n, nullptr, frames, n_frames, ws, ws_bytes, save != 0, &L, &c);
    if (rc != GFTORF_OK) return rc;
    if (!delta) return fail(GFTORF_EINVAL, "NULL pointer");
    (void)hipGetLastError();
    const hipError_t e = gft::mlp::launch_fwd(L, c, delta, save != 0, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GFTORF_OK : hip_fail(e, "gftorf_mlp_fwd_frames");
}

int gftorf_mlp_bwd_frames(const gftorf_mlp_config* cfg, const float* params, const float* x0,
                          int64_t n, const gftorf_frame* frames, int32_t n_frames,
                          const float* d_delta, float* d_params, float* d_x0, int32_t accumulate_x0,
                          void* ws, size_t ws_bytes, void* stream) {
    gft::mlp::Layout L;
    gft::mlp::Call c;
    if (!frames) return fail(GFTORF_EINVAL, "NULL pointer");
    const int rc = mlp_call(cfg, params, x0, n, nullptr, frames, n_frames, ws, ws_bytes, true, &L, &c);
    if (rc != GFTORF_OK) return rc;
    if (!d_delta || !d_params) return fail(GFTORF_EINVAL, "NULL pointer");
    (void)hipGetLastError();
    const hipError_t e = gft::mlp::launch_bwd(L, c, d_delta, d_params, d_x0, accumulate_x0 != 0,
                                              static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GFTORF_OK : hip_fail(e, "gftorf_mlp_bwd_frames");
}

namespace {
int blend_args(int32_t n_steps, int64_t n, const gftorf_frame* frames, int32_t n_frames,
               const int32_t* anchors, gft::mlp::Blend* b) {
    if (!frames || !anchors || n < 0 || n_steps < 1 || n_frames < 0 ||
        n_frames > gft::mlp::kMaxBlendFrames)
        return fail(GFTORF_EINVAL, "bad blend arguments (1 <= n_steps, 0 <= n_frames <= 256)");
    for (int f = 0; f < 2 * n_frames; ++f)
        if (anchors[f] < 0 || anchors[f] >= n_steps)
            return fail(GFTORF_EINVAL, "anchor step out of range");
    for (int f = 0; f < 2 * gft::mlp::kMaxBlendFrames; ++f) b->anchors[f] = f < 2 * n_frames ? anchors[f] : 0;
    b->n_frames = n_frames;
    b->n_steps = n_steps;
    b->n = n;
    return GFTORF_OK;
}
}  // namespace

int gftorf_blend_offsets(const float* delta_steps, int32_t n_steps, int64_t n,
                         const gftorf_frame* frames, int32_t n_frames, const int32_t* anchors,
                         float* delta_frames, void* stream) {
    gft::mlp::Blend b;
    const int rc = blend_args(n_steps, n, frames, n_frames, anchors, &b);
    if (rc != GFTORF_OK) return rc;
    if ((!delta_steps || !delta_frames) && n > 0) return fail(GFTORF_EINVAL, "NULL pointer");
    (void)hipGetLastError();
    const hipError_t e = gft::mlp::launch_blend(b, delta_steps, frames, delta_frames, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GFTORF_OK : hip_fail(e, "gftorf_blend_offsets");
}

int gftorf_blend_offsets_bwd(const float* d_frames, int32_t n_frames, int64_t n,
                             const gftorf_frame* frames, const int32_t* anchors, int32_t n_steps,
                             float* d_steps, void* stream) {
    gft::mlp::Blend b;
    const int rc = blend_args(n_steps, n, frames, n_frames, anchors, &b);
    if (rc != GFTORF_OK) return rc;
    if ((!d_frames || !d_steps) && n > 0) return fail(GFTORF_EINVAL, "NULL pointer");
    (void)hipGetLastError();
    const hipError_t e = gft::mlp::launch_blend_bwd(b, d_frames, frames, d_steps, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GFTORF_OK : hip_fail(e, "gftorf_blend_offsets_bwd");
}

int gftorf_fill_f32(float* p, float value, int64_t n, void* stream) {
    if (!p && n > 0) return fail(GFTORF_EINVAL, "NULL pointer");
    (void)hipGetLastError();
    gft::launch_fill_f32(p, value, n, static_cast<hipStream_t>(stream));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GFTORF_OK : hip_fail(e, "gftorf_fill_f32");
}

int gftorf_graph_begin(void* stream) {
    hipError_t e = hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal);
    return e == hipSuccess ? GFTORF_OK : hip_fail(e, "gftorf_graph_begin");
}

int gftorf_graph_end(void* stream, void** graph_exec) {
    if (!graph_exec) return fail(GFTORF_EINVAL, "graph_exec is NULL");
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(static_cast<hipStream_t>(stream), &graph);
    if (e != hipSuccess) return hip_fail(e, "gftorf_graph_end (capture)");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "gftorf_graph_end (instantiate)");
    *graph_exec = exec;
    return GFTORF_OK;
}

int gftorf_graph_launch(void* graph_exec, void* stream) {
    if (!graph_exec) return fail(GFTORF_EINVAL, "graph_exec is NULL");
    hipError_t e = hipGraphLaunch(static_cast<hipGraphExec_t>(graph_exec), static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GFTORF_OK : hip_fail(e, "gftorf_graph_launch");
}

int gftorf_graph_destroy(void* graph_exec) {
    if (!graph_exec) return GFTORF_OK;
    hipError_t e = hipGraphExecDestroy(static_cast<hipGraphExec_t>(graph_exec));
    return e == hipSuccess ? GFTORF_OK : hip_fail(e, "gftorf_graph_destroy");
}

const char* gftorf_strerror(int code) {
    switch (code) {
        case GFTORF_OK: return "ok";
        case GFTORF_EINVAL: return "invalid argument";
        case GFTORF_ENOWS: return "workspace too small";
        case GFTORF_EHIP: return "HIP runtime error";
        case GFTORF_EOVERFLOW: return "pair capacity overflow";
        default: return "unknown error";
    }
}

const char* gftorf_last_error(void) { return g_err.c_str(); }

int gftorf_version(void) { return 1; }

}  // extern "C"

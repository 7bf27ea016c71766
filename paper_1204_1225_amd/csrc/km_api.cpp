// C ABI of libkirchhoff.so (declared in include/kirchhoff.h): argument
// validation, tile-shape choice, the shape-class tuning cache and the batched
// hipGraph handle.  All device work is in the km_*.hip kernel files.
#include "kirchhoff.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "km_kernels.h"

namespace {

thread_local std::string g_last_error;

km_status fail(km_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

km_status hip_fail(hipError_t e, const char* what) {
    return fail(KM_E_HIP, "%s: %s (%d)", what, hipGetErrorString(e), static_cast<int>(e));
}

// Failure injection for tests of the error path: with KM_FAULT_INJECT=launch
// in the environment every kernel launch of the library reports a HIP launch
// failure instead of launching (nothing runs; outputs are untouched).
bool inject_launch_failure() {
    const char* v = std::getenv("KM_FAULT_INJECT");
    return v && std::strcmp(v, "launch") == 0;
}

// The status of a launch that is about to happen: KM_E_HIP when failures are injected.
km_status injected(const char* what) {
    return inject_launch_failure() ? fail(KM_E_HIP, "%s: launch failure injected (KM_FAULT_INJECT=launch)", what)
                                   : KM_OK;
}

constexpr int kMaxLds = 160 * 1024;  // LDS per workgroup on gfx950
constexpr int kMaxTracesPerBlock = 32;
constexpr int kTailPad = 2;

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

km_status check_traces(const km_traces* t, bool need_samples, const char* who) {
    if (!t) return fail(KM_E_INVALID, "%s: traces is NULL", who);
    if (t->n_traces < 0) return fail(KM_E_INVALID, "%s: n_traces < 0", who);
    if (t->n_samples < 0) return fail(KM_E_INVALID, "%s: n_samples < 0", who);
    if (t->n_samples > km_max_samples())
        return fail(KM_E_UNSUPPORTED, "%s: n_samples %d exceeds km_max_samples() = %d", who, t->n_samples,
                    km_max_samples());
    if (t->trace_stride < t->n_samples) return fail(KM_E_INVALID, "%s: trace_stride < n_samples", who);
    if (t->dtype != KM_F32 && t->dtype != KM_BF16 && t->dtype != KM_F16)
        return fail(KM_E_INVALID, "%s: unknown dtype %d", who, t->dtype);
    if (!(t->dt > 0.0) || !std::isfinite(t->dt)) return fail(KM_E_INVALID, "%s: dt must be finite and > 0", who);
    if (!std::isfinite(t->t_first)) return fail(KM_E_INVALID, "%s: t_first must be finite", who);
    if (std::fabs(t->t_first / t->dt) > 1.0e7) return fail(KM_E_UNSUPPORTED, "%s: |t_first / dt| > 1e7", who);
    if (t->dtype == KM_F32 && t->scale) return fail(KM_E_INVALID, "%s: scale must be NULL for KM_F32", who);
    if (t->n_traces > 0) {
        if (!t->src || !t->rec || !t->bin) return fail(KM_E_INVALID, "%s: src, rec and bin must be non-NULL", who);
        if (!aligned(t->src, 4) || !aligned(t->rec, 4) || !aligned(t->bin, 4))
            return fail(KM_E_INVALID, "%s: src, rec, bin must be 4-byte aligned", who);
        if (need_samples && t->n_samples > 0) {
            if (!t->data) return fail(KM_E_INVALID, "%s: data is NULL", who);
            if (!aligned(t->data, t->dtype == KM_F32 ? 4 : 2))
                return fail(KM_E_INVALID, "%s: data is misaligned for its dtype", who);
            if (t->trace_stride > 0 && t->n_traces > INT64_MAX / t->trace_stride)
                return fail(KM_E_INVALID, "%s: n_traces * trace_stride overflows", who);
        }
        if (t->scale && !aligned(t->scale, 4)) return fail(KM_E_INVALID, "%s: scale misaligned", who);
    }
    return KM_OK;
}

km_status check_grid(const km_grid* g, const km_traveltime* tt, const km_weight* w, const char* who) {
    if (!g || !tt || !w) return fail(KM_E_INVALID, "%s: grid, traveltime and weight must be non-NULL", who);
    if (g->nx < 0 || g->ny < 0 || g->nz < 0 || g->n_bins < 0) return fail(KM_E_INVALID, "%s: negative grid size", who);
    if (static_cast<int64_t>(g->nx) * g->ny >= (int64_t(1) << 31))
        return fail(KM_E_UNSUPPORTED, "%s: nx * ny must be < 2^31", who);
    if (g->n_bins > 65535) return fail(KM_E_UNSUPPORTED, "%s: n_bins > 65535", who);
    if (w->kind != KM_W_UNIT && w->kind != KM_W_COSCOS_OVER_TT)
        return fail(KM_E_INVALID, "%s: unknown weight kind %d", who, w->kind);
    if (tt->time_precision != KM_TIME_FP32 && tt->time_precision != KM_TIME_EXTENDED)
        return fail(KM_E_INVALID, "%s: unknown time precision %d", who, tt->time_precision);
    const bool empty = g->nx == 0 || g->ny == 0 || g->nz == 0 || g->n_bins == 0;
    if (!empty) {
        if (!g->x || !g->y) return fail(KM_E_INVALID, "%s: x and y must be non-NULL", who);
        if (!tt->t0sq || !tt->s2 || !tt->r2) return fail(KM_E_INVALID, "%s: t0sq, s2, r2 must be non-NULL", who);
        if (!aligned(g->x, 4) || !aligned(g->y, 4) || !aligned(tt->t0sq, 4) || !aligned(tt->s2, 4) ||
            !aligned(tt->r2, 4))
            return fail(KM_E_INVALID, "%s: grid / table pointers must be 4-byte aligned", who);
    }
    return KM_OK;
}

bool grid_empty(const km_grid* g) { return g->nx == 0 || g->ny == 0 || g->nz == 0 || g->n_bins == 0; }

// Base parameters (independent of the tile shape).
km::Params base_params(const km_traces* t, const km_grid* g, const km_traveltime* tt, const km_weight* w,
                       float* image, int accumulate) {
    km::Params P{};
    P.data = t->data;
    P.scale = t->scale;
    P.src = t->src;
    P.rec = t->rec;
    P.bin = t->bin;
    P.n_traces = t->n_traces;
    P.stride = t->trace_stride;
    P.nt = t->n_samples;
    P.dtype = t->dtype;
    P.x = g->x;
    P.y = g->y;
    P.nx = g->nx;
    P.ny = g->ny;
    P.nz = g->nz;
    P.n_bins = g->n_bins;
    P.t0sq = tt->t0sq;
    P.s2 = tt->s2;
    P.r2 = tt->r2;
    P.inv_dt2 = 1.0 / (t->dt * t->dt);
    P.wscale = P.inv_dt2 * P.inv_dt2;
    P.has_tf = t->t_first != 0.0 ? 1 : 0;
    P.tf_off = static_cast<float>(km::kLead - t->t_first / t->dt);
    P.tf_off_d = km::kLead - t->t_first / t->dt;
    P.inv_dt = 1.0 / t->dt;
    P.prec = tt->time_precision == KM_TIME_EXTENDED ? 1 : 0;
    P.weight = w->kind;
    P.image = image;
    P.accumulate = accumulate ? 1 : 0;
    P.lt = (t->n_samples + km::kLead + kTailPad + 3) / 4 * 4;
    return P;
}

// Traces per LDS block for a shape's budget; 0 if even one row does not fit.
int traces_per_block(int lt, int budget, int ks, int row_bytes_per_sample) {
    const int64_t fixed = static_cast<int64_t>(16) * ks * 4 + (ks > 0 ? km::kBoxFloats * 4 : 0);
    const int64_t per = static_cast<int64_t>(lt) * row_bytes_per_sample + 16;
    int64_t tb = (budget - fixed) / per;
    if (tb < 1 && fixed + per <= kMaxLds) tb = 1;
    return static_cast<int>(std::min<int64_t>(tb, kMaxTracesPerBlock));
}

// Migrate blocks: at most kMigrateSlots traces, and the shape's LDS budget
// less the fixed part for their time windows (2 floats per staged sample, 1
// for table traveltimes, half as many bytes with 16-bit staging);
// at least one whole record (samples -1 .. nt + 1) must fit, with fewer
// slots for the longest records.  Sets P.tb and P.cap (floats); false if a
// record does not fit in LDS.
constexpr int kMigrateSlots = 128;
bool migrate_block_params(km::Params& P, int budget, int ks) {
    // square-root times stage (sample, difference) pairs, table times samples,
    // 16-bit staging packed pairs of 16-bit samples and 16-bit samples (half
    // as many bytes), anti-aliasing float64 running sums over nt + 4 max_half
    // + 9 positions
    const int64_t nt = P.nt;
    const int64_t need = (P.aa_max > 0 ? 2 * (nt + 4 * P.aa_max + 9)
                          : P.ttab   ? (P.s16 ? (nt + 4) / 2 : nt + 3)
                                     : (P.s16 ? nt + 2 : 2 * (nt + 2))) + 3 & ~int64_t{3};
    for (int tb = kMigrateSlots; tb >= 1; tb /= 2) {
        const int64_t fixed = static_cast<int64_t>(km::migrate_lds_words(0, tb, ks));
        const int64_t cap = std::max<int64_t>((budget / 4 - fixed) & ~int64_t{3}, need);
        if ((fixed + cap) * 4 <= kMaxLds) {
            P.tb = tb;
            P.cap = static_cast<int>(cap);
            return true;
        }
    }
    return false;
}

int shape_count(int op) { return op == 0 ? km::migrate_shape_count() : km::demigrate_shape_count(); }

// A tile is a compiled shape and a runtime variant of it, encoded as
// shape + kTileLevelStride * level.  Migrate levels scale the LDS budget of the
// trace block (traces per block): 1, 0.5, 1.5, 2 times the shape's, and levels
// 4 and 5 stage 16-bit traces as their 16-bit storage (the S16 kernels) with 1
// and 2 times the budget: twice the samples per byte of float staging.
// Demigrate level 0 takes as many trace quads per workgroup as the shape's
// budget and template allow; level L >= 1 takes L quads (L <= the shape's
// quads).
constexpr int kTileLevelStride = 64;
constexpr int kMigrateLevels = 6;
constexpr int kDemigrateLevels = 4;
constexpr double kMigrateBudgetScale[kMigrateLevels] = {1.0, 0.5, 1.5, 2.0, 1.0, 2.0};
constexpr int kMigrateLds16[kMigrateLevels] = {0, 0, 0, 0, 1, 1};
// the float-staging level of a 16-bit staging level's budget
constexpr int kMigrateFloatLevel[kMigrateLevels] = {0, 1, 2, 3, 0, 3};

int level_count(int op) { return op == 0 ? kMigrateLevels : kDemigrateLevels; }

bool decode_tile(int op, int tile, int* shape, int* level) {
    if (tile < 0) return false;
    *shape = tile % kTileLevelStride;
    *level = tile / kTileLevelStride;
    if (*shape >= shape_count(op) || *level >= level_count(op)) return false;
    if (op == 1 && *level > 0 && *level > km::demigrate_shape(*shape).max_quads) return false;
    return true;
}

km_status shape_params(int op, int tile, km::Params& P) {
    int shape = 0, level = 0;
    if (!decode_tile(op, tile, &shape, &level)) return fail(KM_E_INVALID, "tile %d is not a tile of op %d", tile, op);
    const km::TileShape& S = op == 0 ? km::migrate_shape(shape) : km::demigrate_shape(shape);
    if (op == 0) {
        P.s16 = kMigrateLds16[level];
        if (P.s16 && (P.dtype == km::F32 || P.aa_max > 0 || P.prec))
            return fail(KM_E_UNSUPPORTED,
                        "tile %d stages 16-bit traces: it needs KM_BF16 or KM_F16 traces, float32 time precision "
                        "and no anti-alias filter", tile);
        const int budget = static_cast<int>(std::min<double>(kMaxLds, S.lds_budget * kMigrateBudgetScale[level]));
        if (!migrate_block_params(P, budget, S.depth_slots)) P.tb = 0;
    } else {
        // float64 rows; the four groups of a wavefront take four traces, so
        // whole quads of traces keep every group busy
        // (anti-aliased rows are longer: the budget grows with them, keeping whole quads)
        const int extra = P.aa_max > 0 ? 4 * 8 * (P.lt - (P.nt + km::kLead + kTailPad + 3) / 4 * 4) : 0;
        P.tb = traces_per_block(P.lt, S.lds_budget + extra, 0, 8);
        if (S.max_quads > 0) P.tb = std::min(P.tb, 4 * S.max_quads);
        if (level > 0) P.tb = std::min(P.tb, 4 * level);
        if (P.tb >= 4) P.tb &= ~3;
    }
    if (P.tb < 1) return fail(KM_E_UNSUPPORTED, "record of %d samples does not fit in LDS", P.nt);
    const int zchunk = 16 * S.depth_slots;
    P.n_zchunks = (P.nz + zchunk - 1) / zchunk;
    if (P.n_zchunks > 65535) return fail(KM_E_UNSUPPORTED, "nz = %d needs more than 65535 depth chunks", P.nz);
    const int cols = S.waves * S.column_groups * 4;
    const int ncol = P.nx * P.ny;
    P.n_coltiles = (ncol + cols - 1) / cols;
    return KM_OK;
}

// ---- tuning cache ----------------------------------------------------------
// Keyed by (GPU architecture, op, dtype, traveltime kind, time precision,
// depth bucket nz / 128, sample bucket n_samples / 512); persisted as JSON to
// the file named by the KM_TUNE_CACHE environment variable (read on first
// use, rewritten after every record).
struct TuneKey {
    std::string arch;
    int op, dtype, kind, prec, nzb, ntb;
    bool operator<(const TuneKey& o) const {
        return std::tie(arch, op, dtype, kind, prec, nzb, ntb) <
               std::tie(o.arch, o.op, o.dtype, o.kind, o.prec, o.nzb, o.ntb);
    }
};

struct TuneEntry {
    int tile;
    float ms;
};

std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;
bool g_tune_loaded = false;

// Architecture of the current device ("gfx950"), or "unknown" without one.
std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

TuneKey tune_key(int op, int dtype, int kind, int prec, int nz, int nt) {
    return TuneKey{device_arch(), op, dtype, kind, prec, (nz + 127) / 128, (nt + 511) / 512};
}

const char* tune_cache_path() {
    const char* p = std::getenv("KM_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

// The value of "name": in one JSON object's text (our own flat format).
bool json_field(const std::string& obj, const char* name, std::string* out) {
    const std::string k = std::string("\"") + name + "\"";
    size_t i = obj.find(k);
    if (i == std::string::npos) return false;
    i = obj.find(':', i + k.size());
    if (i == std::string::npos) return false;
    ++i;
    while (i < obj.size() && (obj[i] == ' ' || obj[i] == '\t' || obj[i] == '\n')) ++i;
    if (i < obj.size() && obj[i] == '"') {
        const size_t j = obj.find('"', i + 1);
        if (j == std::string::npos) return false;
        *out = obj.substr(i + 1, j - i - 1);
        return true;
    }
    size_t j = i;
    while (j < obj.size() && obj[j] != ',' && obj[j] != '}' && obj[j] != '\n') ++j;
    *out = obj.substr(i, j - i);
    return !out->empty();
}

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = tune_cache_path();
    if (!path) return;
    FILE* f = std::fopen(path, "rb");
    if (!f) return;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
    std::fclose(f);
    size_t pos = text.find("\"entries\"");
    while (pos != std::string::npos) {
        const size_t a = text.find('{', pos);
        if (a == std::string::npos) break;
        const size_t b = text.find('}', a);
        if (b == std::string::npos) break;
        const std::string obj = text.substr(a, b - a + 1);
        pos = b + 1;
        std::string v[9];
        const char* names[9] = {"arch", "op", "dtype", "kind", "precision", "nz_bucket", "nt_bucket", "tile", "ms"};
        bool ok = true;
        for (int k = 0; k < 9 && ok; ++k) ok = json_field(obj, names[k], &v[k]);
        if (!ok) continue;
        TuneKey key{v[0], std::atoi(v[1].c_str()), std::atoi(v[2].c_str()), std::atoi(v[3].c_str()),
                    std::atoi(v[4].c_str()), std::atoi(v[5].c_str()), std::atoi(v[6].c_str())};
        int shape = 0, level = 0;
        const int tile = std::atoi(v[7].c_str());
        if ((key.op == 0 || key.op == 1) && decode_tile(key.op, tile, &shape, &level))
            g_tune[key] = TuneEntry{tile, static_cast<float>(std::atof(v[8].c_str()))};
    }
}

void tune_save_locked() {
    const char* path = tune_cache_path();
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    std::fprintf(f, "{\n  \"format\": \"km_tune_cache\",\n  \"version\": 1,\n  \"entries\": [");
    bool first = true;
    for (const auto& kv : g_tune) {
        const TuneKey& k = kv.first;
        std::fprintf(f,
                     "%s\n    {\"arch\": \"%s\", \"op\": %d, \"dtype\": %d, \"kind\": %d, \"precision\": %d, "
                     "\"nz_bucket\": %d, \"nt_bucket\": %d, \"tile\": %d, \"ms\": %.4f}",
                     first ? "" : ",", k.arch.c_str(), k.op, k.dtype, k.kind, k.prec, k.nzb, k.ntb, kv.second.tile,
                     static_cast<double>(kv.second.ms));
        first = false;
    }
    std::fprintf(f, "\n  ]\n}\n");
    const bool ok = std::fclose(f) == 0;
    if (ok) std::rename(tmp.c_str(), path);
}

// Traveltime kinds of the cache key.
enum { KIND_DSR = 0, KIND_TABLE = 1, KIND_AA = 2, KIND_LTABLE = 3 };

// Untuned choice: the shapes measured fastest on the 3D survey (migrate:
// 8 waves x 4 column groups x 8 slots; demigrate: 8 waves x 4 slots x 1
// trace quad, and 16 waves x 8 slots x 3 quads with table traveltimes, whose
// table gathers favour more traces per workgroup).  With the anti-alias
// filter: migrate 16 waves x 4 column groups x 8 slots (the largest trace
// blocks), demigrate 8 waves x 4 slots x 1 quad.  With laterally varying
// tables (16 reads per pair): migrate 4 waves x 3 column groups x 16 slots,
// demigrate 8 waves x 8 slots x 3 quads.
int default_tile(int op, int kind) {
    if (op == 0) return kind == KIND_AA ? 1 : kind == KIND_LTABLE ? 3 : 2;
    if (kind == KIND_AA) return 3;
    if (kind == KIND_LTABLE) return 4;
    return kind == KIND_TABLE ? 1 : 3;
}

// Whether a tile can run problems of a class: a tile of op, and a 16-bit
// staging level only for 16-bit traces with float32 time and no anti-alias
// filter.
bool tile_applies(int op, int tile, int dtype, int kind, int prec) {
    int shape = 0, level = 0;
    if (!decode_tile(op, tile, &shape, &level)) return false;
    if (op == 0 && kMigrateLds16[level]) return dtype != KM_F32 && prec != KM_TIME_EXTENDED && kind != KIND_AA;
    return true;
}

// The caller's tile, else the tuned tile of this problem's class (if it still
// applies: a cache file may come from another build), else the default.
km_status pick_tile(int op, int tile, int dtype, int kind, int prec, int nz, int nt, int* out) {
    if (tile >= 0) {
        int shape = 0, level = 0;
        if (!decode_tile(op, tile, &shape, &level))
            return fail(KM_E_INVALID, "tile %d out of range (shape < %d, level < %d)", tile, shape_count(op),
                        level_count(op));
        *out = tile;
        return KM_OK;
    }
    {
        const TuneKey key = tune_key(op, dtype, kind, prec, nz, nt);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end() && tile_applies(op, it->second.tile, dtype, kind, prec)) {
            *out = it->second.tile;
            return KM_OK;
        }
    }
    *out = default_tile(op, kind);
    return KM_OK;
}

// The node grid of laterally varying tables (a km_ltable without its arrays).
struct Lateral {
    int32_t n_gx, n_gy;
    double gx0, gy0, gdx, gdy;
};

km_status run_op(int op, const km_traces* t, const km_grid* g, const km_traveltime* tt, const km_weight* w,
                 float* image, int accumulate, int tile, hipStream_t s, const km_ttable* tab = nullptr,
                 const km_antialias* aa = nullptr, const Lateral* lat = nullptr) {
    km::Params P = base_params(t, g, tt, w, image, accumulate);
    if (aa) {
        P.aa_dx = static_cast<float>(aa->dx);
        P.aa_dy = static_cast<float>(aa->dy);
        P.aa_max = aa->max_half;
        // demigrate rows: samples -aa_lead .. nt + aa_lead - 1 (the dual of the
        // double running sum reaches 2 max_half + 4 past either end)
        P.aa_lead = 2 * aa->max_half + 5;
        P.lt = (t->n_samples + 2 * P.aa_lead + 3) / 4 * 4;
    }
    if (tab) {
        P.ttab = tab->t;
        P.n_h = tab->n_h;
        P.inv_dh = static_cast<float>(1.0 / tab->dh);
        P.inv_dh_d = 1.0 / tab->dh;
        P.t0sq = nullptr;
        P.s2 = nullptr;
        P.r2 = tab->r2;
        P.tamp = tab->amp;
        P.weight = KM_W_UNIT;
        // < 2^31: checked with the table
        P.ttab_bytes = static_cast<uint32_t>(int64_t{4} * tab->n_h * g->nz * (lat ? int64_t{lat->n_gx} * lat->n_gy : 1));
    }
    if (tab && lat) {
        const int32_t node = tab->n_h * g->nz;  // < 2^29: checked with the whole table
        P.n_gx = lat->n_gx;
        P.n_gy = lat->n_gy;
        P.ldx = lat->n_gx > 1 ? node : 0;
        P.ldy = lat->n_gy > 1 ? lat->n_gx * node : 0;
        P.gx0 = lat->gx0;
        P.gy0 = lat->gy0;
        P.gdx = lat->gdx;
        P.gdy = lat->gdy;
    }
    km_status st = shape_params(op, tile, P);
    if (st != KM_OK) return st;
    const int shape = tile % kTileLevelStride;
    if (op == 1 && (P.n_traces + P.tb - 1) / P.tb > INT32_MAX)
        return fail(KM_E_UNSUPPORTED, "kirchhoff_demigrate: too many trace blocks");
    if (op == 0 && P.n_traces > INT32_MAX)  // block slots record trace indices within a bin as int32
        return fail(KM_E_UNSUPPORTED, "kirchhoff_migrate: more than 2^31 - 1 traces");
    st = injected(op == 0 ? "migrate launch" : "demigrate launch");
    if (st != KM_OK) return st;
    hipError_t e = op == 0 ? km::launch_migrate(shape, P, s) : km::launch_demigrate(shape, P, s);
    if (e != hipSuccess) return hip_fail(e, op == 0 ? "migrate launch" : "demigrate launch");
    return KM_OK;
}

// Image zero fill for empty problems (nothing to evaluate, overwrite semantics).
km_status zero_floats(float* p, int64_t n, hipStream_t s) {
    if (n <= 0) return KM_OK;
    const km_status st = injected("zero fill");
    if (st != KM_OK) return st;
    const hipError_t e = km::launch_axpby(0.0f, p, 0.0f, p, n, s);
    return e == hipSuccess ? KM_OK : hip_fail(e, "zero fill");
}

km_status migrate_impl(const km_traces* traces, const km_grid* grid, const km_traveltime* tt, const km_weight* weight,
                       float* image, int32_t accumulate, int32_t tile, void* stream, const km_ttable* tab,
                       const km_antialias* aa = nullptr, const Lateral* lat = nullptr) {
    km_status st = check_traces(traces, true, "kirchhoff_migrate");
    if (st != KM_OK) return st;
    st = check_grid(grid, tt, weight, "kirchhoff_migrate");
    if (st != KM_OK) return st;
    if (grid_empty(grid)) return KM_OK;
    if (!image || !aligned(image, 4)) return fail(KM_E_INVALID, "kirchhoff_migrate: image is NULL or misaligned");
    int shape = 0;
    st = pick_tile(0, tile, traces->dtype, lat ? KIND_LTABLE : tab ? KIND_TABLE : aa ? KIND_AA : KIND_DSR,
                   tt->time_precision, grid->nz, traces->n_samples, &shape);
    if (st != KM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (traces->n_traces == 0 && !accumulate)
        return zero_floats(image, static_cast<int64_t>(grid->n_bins) * grid->ny * grid->nx * grid->nz, s);
    return run_op(0, traces, grid, tt, weight, image, accumulate, shape, s, tab, aa, lat);
}

km_status demigrate_impl(const float* image, const km_grid* grid, const km_traveltime* tt, const km_weight* weight,
                         const km_traces* out, int32_t accumulate, int32_t tile, void* stream, const km_ttable* tab,
                         const km_antialias* aa = nullptr, const Lateral* lat = nullptr) {
    km_status st = check_traces(out, true, "kirchhoff_demigrate");
    if (st != KM_OK) return st;
    if (out->dtype != KM_F32)
        return fail(KM_E_UNSUPPORTED, "kirchhoff_demigrate: output traces must be KM_F32");
    st = check_grid(grid, tt, weight, "kirchhoff_demigrate");
    if (st != KM_OK) return st;
    if (out->n_traces == 0 || out->n_samples == 0) return KM_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (grid_empty(grid)) {
        if (accumulate) return KM_OK;
        if (out->trace_stride != out->n_samples)
            return fail(KM_E_UNSUPPORTED, "kirchhoff_demigrate: empty grid with strided output");
        return zero_floats(static_cast<float*>(out->data), out->n_traces * out->trace_stride, s);
    }
    if (!image || !aligned(image, 4)) return fail(KM_E_INVALID, "kirchhoff_demigrate: image is NULL or misaligned");
    int shape = 0;
    st = pick_tile(1, tile, out->dtype, lat ? KIND_LTABLE : tab ? KIND_TABLE : aa ? KIND_AA : KIND_DSR,
                   tt->time_precision, grid->nz, out->n_samples, &shape);
    if (st != KM_OK) return st;
    return run_op(1, out, grid, tt, weight, const_cast<float*>(image), accumulate, shape, s, tab, aa, lat);
}

// Anti-alias filter options.
km_status check_antialias(const km_antialias* aa, const char* who) {
    if (!aa) return fail(KM_E_INVALID, "%s: anti-alias options are NULL", who);
    if (!(aa->dx >= 0.0) || !(aa->dy >= 0.0) || !std::isfinite(aa->dx) || !std::isfinite(aa->dy))
        return fail(KM_E_INVALID, "%s: dx and dy must be finite and >= 0", who);
    if (aa->max_half < 1 || aa->max_half > km::kAAMaxHalf)
        return fail(KM_E_INVALID, "%s: max_half must be in [1, %d]", who, km::kAAMaxHalf);
    return KM_OK;
}

km_status check_antialias_tt(const km_traveltime* tt, const char* who) {
    if (tt && tt->time_precision == KM_TIME_EXTENDED)
        return fail(KM_E_UNSUPPORTED, "%s: the anti-alias operators evaluate float32 times only", who);
    return KM_OK;
}

// Table traveltimes: validate the table, then run the shared path with the
// table in place of t0sq / s2 (only r2 of the traveltime struct is read).
km_status check_table(const km_ttable* tab, const km_grid* grid, const char* who) {
    if (!tab) return fail(KM_E_INVALID, "%s: table is NULL", who);
    if (tab->n_h < 2) return fail(KM_E_INVALID, "%s: n_h < 2", who);
    if (!(tab->dh > 0.0) || !std::isfinite(tab->dh)) return fail(KM_E_INVALID, "%s: dh must be finite and > 0", who);
    if (grid && static_cast<int64_t>(tab->n_h) * grid->nz >= (int64_t(1) << 29))
        return fail(KM_E_UNSUPPORTED, "%s: n_h * nz must be < 2^29", who);
    if (grid && !grid_empty(grid)) {
        if (!tab->t || !tab->r2) return fail(KM_E_INVALID, "%s: t and r2 must be non-NULL", who);
        if (!aligned(tab->t, 4) || !aligned(tab->r2, 4) || !aligned(tab->amp, 4))
            return fail(KM_E_INVALID, "%s: t, r2 or amp misaligned", who);
    }
    return KM_OK;
}

// Laterally varying tables: the node grid, then the table as check_table
// sees it (the node tables together must stay below 2^29 floats: the kernels
// read them through one buffer whose byte offsets are 32-bit signed values).
km_status check_ltable(const km_ltable* lt, const km_grid* grid, const char* who, km_ttable* tab, Lateral* lat) {
    if (!lt) return fail(KM_E_INVALID, "%s: table is NULL", who);
    if (lt->n_gx < 1 || lt->n_gy < 1) return fail(KM_E_INVALID, "%s: n_gx and n_gy must be >= 1", who);
    if (!std::isfinite(lt->gx0) || !std::isfinite(lt->gy0))
        return fail(KM_E_INVALID, "%s: gx0 and gy0 must be finite", who);
    if ((lt->n_gx > 1 && !(lt->gdx > 0.0 && std::isfinite(lt->gdx))) ||
        (lt->n_gy > 1 && !(lt->gdy > 0.0 && std::isfinite(lt->gdy))))
        return fail(KM_E_INVALID, "%s: gdx (gdy) must be finite and > 0 when n_gx (n_gy) > 1", who);
    *tab = km_ttable{lt->n_h, lt->dh, lt->t, lt->r2, lt->time_precision, lt->amp};
    const km_status st = check_table(tab, grid, who);
    if (st != KM_OK) return st;
    if (grid && static_cast<int64_t>(lt->n_gx) * lt->n_gy * lt->n_h * grid->nz >= (int64_t(1) << 29))
        return fail(KM_E_UNSUPPORTED, "%s: n_gx * n_gy * n_h * nz must be < 2^29", who);
    *lat = Lateral{lt->n_gx, lt->n_gy, lt->gx0, lt->gy0, lt->n_gx > 1 ? lt->gdx : 1.0, lt->n_gy > 1 ? lt->gdy : 1.0};
    return KM_OK;
}

}  // namespace

// Status and per-thread message for the C ABI calls defined in other files.
km_status km_set_error(km_status st, const char* msg) { return fail(st, "%s", msg); }

extern "C" {

int km_abi_version(void) { return KM_ABI_VERSION; }

const char* km_last_error(void) { return g_last_error.c_str(); }

// one float64 accumulator row (demigrate), its geometry and the chunk tables fit in 160 KiB
int32_t km_max_samples(void) { return 20000; }

km_status kirchhoff_migrate(const km_traces* traces, const km_grid* grid, const km_traveltime* tt,
                            const km_weight* weight, float* image, int32_t accumulate, int32_t tile, void* stream) {
    return migrate_impl(traces, grid, tt, weight, image, accumulate, tile, stream, nullptr);
}

km_status kirchhoff_demigrate(const float* image, const km_grid* grid, const km_traveltime* tt,
                              const km_weight* weight, const km_traces* out, int32_t accumulate, int32_t tile,
                              void* stream) {
    return demigrate_impl(image, grid, tt, weight, out, accumulate, tile, stream, nullptr);
}

km_status kirchhoff_migrate_table(const km_traces* traces, const km_grid* grid, const km_ttable* tab, float* image,
                                  int32_t accumulate, int32_t tile, void* stream) {
    km_status st = check_table(tab, grid, "kirchhoff_migrate_table");
    if (st != KM_OK) return st;
    const km_traveltime tt{tab->r2, tab->r2, tab->r2, tab->time_precision};
    const km_weight w{KM_W_UNIT};
    return migrate_impl(traces, grid, &tt, &w, image, accumulate, tile, stream, tab);
}

km_status kirchhoff_demigrate_table(const float* image, const km_grid* grid, const km_ttable* tab,
                                    const km_traces* out, int32_t accumulate, int32_t tile, void* stream) {
    km_status st = check_table(tab, grid, "kirchhoff_demigrate_table");
    if (st != KM_OK) return st;
    const km_traveltime tt{tab->r2, tab->r2, tab->r2, tab->time_precision};
    const km_weight w{KM_W_UNIT};
    return demigrate_impl(image, grid, &tt, &w, out, accumulate, tile, stream, tab);
}

km_status kirchhoff_migrate_ltable(const km_traces* traces, const km_grid* grid, const km_ltable* ltab, float* image,
                                   int32_t accumulate, int32_t tile, void* stream) {
    km_ttable tab;
    Lateral lat;
    km_status st = check_ltable(ltab, grid, "kirchhoff_migrate_ltable", &tab, &lat);
    if (st != KM_OK) return st;
    const km_traveltime tt{tab.r2, tab.r2, tab.r2, tab.time_precision};
    const km_weight w{KM_W_UNIT};
    return migrate_impl(traces, grid, &tt, &w, image, accumulate, tile, stream, &tab, nullptr, &lat);
}

km_status kirchhoff_demigrate_ltable(const float* image, const km_grid* grid, const km_ltable* ltab,
                                     const km_traces* out, int32_t accumulate, int32_t tile, void* stream) {
    km_ttable tab;
    Lateral lat;
    km_status st = check_ltable(ltab, grid, "kirchhoff_demigrate_ltable", &tab, &lat);
    if (st != KM_OK) return st;
    const km_traveltime tt{tab.r2, tab.r2, tab.r2, tab.time_precision};
    const km_weight w{KM_W_UNIT};
    return demigrate_impl(image, grid, &tt, &w, out, accumulate, tile, stream, &tab, nullptr, &lat);
}

km_status kirchhoff_migrate_aa(const km_traces* traces, const km_grid* grid, const km_traveltime* tt,
                               const km_weight* weight, const km_antialias* aa, float* image, int32_t accumulate,
                               int32_t tile, void* stream) {
    km_status st = check_antialias(aa, "kirchhoff_migrate_aa");
    if (st == KM_OK) st = check_antialias_tt(tt, "kirchhoff_migrate_aa");
    if (st != KM_OK) return st;
    return migrate_impl(traces, grid, tt, weight, image, accumulate, tile, stream, nullptr, aa);
}

km_status kirchhoff_demigrate_aa(const float* image, const km_grid* grid, const km_traveltime* tt,
                                 const km_weight* weight, const km_antialias* aa, const km_traces* out,
                                 int32_t accumulate, int32_t tile, void* stream) {
    km_status st = check_antialias(aa, "kirchhoff_demigrate_aa");
    if (st == KM_OK) st = check_antialias_tt(tt, "kirchhoff_demigrate_aa");
    if (st != KM_OK) return st;
    return demigrate_impl(image, grid, tt, weight, out, accumulate, tile, stream, nullptr, aa);
}


km_status km_count_contributions(const km_traces* traces, const km_grid* grid, const km_traveltime* tt,
                                 int64_t* counts, void* stream) {
    km_status st = check_traces(traces, false, "km_count_contributions");
    if (st != KM_OK) return st;
    km_weight w{KM_W_UNIT};
    st = check_grid(grid, tt, &w, "km_count_contributions");
    if (st != KM_OK) return st;
    if (!counts || !aligned(counts, 8)) return fail(KM_E_INVALID, "km_count_contributions: counts NULL/misaligned");
    km::Params P = base_params(traces, grid, tt, &w, nullptr, 0);
    if (grid_empty(grid)) { P.nx = P.ny = P.nz = P.n_bins = 0; }
    {
        const km_status ist = injected("count launch");
        if (ist != KM_OK) return ist;
    }
    const hipError_t e = km::launch_count(P, reinterpret_cast<unsigned long long*>(counts),
                                          static_cast<hipStream_t>(stream));
    return e == hipSuccess ? KM_OK : hip_fail(e, "count launch");
}

km_status km_dot_f64(const float* a, const float* b, int64_t n, double* out, void* stream) {
    if (n < 0) return fail(KM_E_INVALID, "km_dot_f64: n < 0");
    if (!out || !aligned(out, 8)) return fail(KM_E_INVALID, "km_dot_f64: out NULL/misaligned");
    if (n > 0 && (!a || !b || !aligned(a, 4) || !aligned(b, 4)))
        return fail(KM_E_INVALID, "km_dot_f64: a, b NULL/misaligned");
    {
        const km_status ist = injected("dot launch");
        if (ist != KM_OK) return ist;
    }
    const hipError_t e = km::launch_dot_f64(a, b, n, out, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? KM_OK : hip_fail(e, "dot launch");
}

km_status km_axpby(double alpha, const float* x, double beta, float* y, int64_t n, void* stream) {
    if (n < 0) return fail(KM_E_INVALID, "km_axpby: n < 0");
    if (n > 0 && (!x || !y || !aligned(x, 4) || !aligned(y, 4)))
        return fail(KM_E_INVALID, "km_axpby: x, y NULL/misaligned");
    if (!std::isfinite(alpha) || !std::isfinite(beta)) return fail(KM_E_INVALID, "km_axpby: non-finite scalar");
    {
        const km_status ist = injected("axpby launch");
        if (ist != KM_OK) return ist;
    }
    const hipError_t e = km::launch_axpby(static_cast<float>(alpha), x, static_cast<float>(beta), y, n,
                                          static_cast<hipStream_t>(stream));
    return e == hipSuccess ? KM_OK : hip_fail(e, "axpby launch");
}

km_status km_trace_filter(const float* in, int64_t in_stride, float* out, int64_t out_stride, int64_t n_traces,
                          int32_t n_samples, const float* taps, int32_t n_taps, int32_t center, int32_t adjoint,
                          void* stream) {
    if (n_traces < 0 || n_samples < 0) return fail(KM_E_INVALID, "km_trace_filter: negative size");
    if (n_taps < 1) return fail(KM_E_INVALID, "km_trace_filter: n_taps < 1");
    if (n_taps > 1024) return fail(KM_E_UNSUPPORTED, "km_trace_filter: n_taps > 1024");
    if (center < 0 || center >= n_taps) return fail(KM_E_INVALID, "km_trace_filter: center outside [0, n_taps)");
    if (in_stride < n_samples || out_stride < n_samples)
        return fail(KM_E_INVALID, "km_trace_filter: stride < n_samples");
    if (n_traces == 0 || n_samples == 0) return KM_OK;
    if (!in || !out || !taps || !aligned(in, 4) || !aligned(out, 4) || !aligned(taps, 4))
        return fail(KM_E_INVALID, "km_trace_filter: in, out, taps NULL/misaligned");
    if (in != out || in_stride != out_stride) {
        const uintptr_t a0 = reinterpret_cast<uintptr_t>(in), b0 = reinterpret_cast<uintptr_t>(out);
        const uintptr_t a1 = a0 + 4 * static_cast<uintptr_t>((n_traces - 1) * in_stride + n_samples);
        const uintptr_t b1 = b0 + 4 * static_cast<uintptr_t>((n_traces - 1) * out_stride + n_samples);
        if (a0 < b1 && b0 < a1) return fail(KM_E_INVALID, "km_trace_filter: in and out overlap");
    }
    if (km::fir_lds_bytes(n_samples, n_taps) > static_cast<size_t>(kMaxLds))
        return fail(KM_E_UNSUPPORTED, "km_trace_filter: %d samples and %d taps do not fit in LDS", n_samples, n_taps);
    {
        const km_status ist = injected("filter launch");
        if (ist != KM_OK) return ist;
    }
    const hipError_t e = km::launch_fir(in, in_stride, out, out_stride, n_traces, n_samples, taps, n_taps, center,
                                        adjoint ? 1 : 0, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? KM_OK : hip_fail(e, "filter launch");
}

km_status km_stack_offsets(const float* image, int32_t n_bins, int64_t n_points, float* stack, void* stream) {
    if (n_bins < 1) return fail(KM_E_INVALID, "km_stack_offsets: n_bins < 1");
    if (n_points < 0) return fail(KM_E_INVALID, "km_stack_offsets: n_points < 0");
    if (n_points == 0) return KM_OK;
    if (!image || !stack || !aligned(image, 4) || !aligned(stack, 4))
        return fail(KM_E_INVALID, "km_stack_offsets: image, stack NULL/misaligned");
    {
        const km_status ist = injected("stack launch");
        if (ist != KM_OK) return ist;
    }
    const hipError_t e = km::launch_stack(image, n_bins, n_points, stack, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? KM_OK : hip_fail(e, "stack launch");
}

km_status km_cig_moveout(const float* image, const km_grid* grid, const float* offsets, int32_t max_lag,
                         int32_t z_lo, int32_t z_hi, float* stack, float* shift, float* peak, float* curvature,
                         void* stream) {
    if (!grid) return fail(KM_E_INVALID, "km_cig_moveout: grid is NULL");
    if (grid->nx < 0 || grid->ny < 0 || grid->nz < 0 || grid->n_bins < 0)
        return fail(KM_E_INVALID, "km_cig_moveout: negative grid size");
    if (static_cast<int64_t>(grid->nx) * grid->ny >= (int64_t(1) << 31))
        return fail(KM_E_UNSUPPORTED, "km_cig_moveout: nx * ny must be < 2^31");
    if (max_lag < 0) return fail(KM_E_INVALID, "km_cig_moveout: max_lag < 0");
    if (max_lag > 256) return fail(KM_E_UNSUPPORTED, "km_cig_moveout: max_lag > 256");
    if (z_lo < 0 || z_hi > grid->nz || z_lo >= z_hi)
        return fail(KM_E_INVALID, "km_cig_moveout: depth window [%d, %d) not inside [0, %d) or empty", z_lo, z_hi,
                    grid->nz);
    if (grid->n_bins < 1) return fail(KM_E_INVALID, "km_cig_moveout: n_bins < 1");
    if (!image || !shift) return fail(KM_E_INVALID, "km_cig_moveout: image and shift must be non-NULL");
    if (!aligned(image, 4) || !aligned(shift, 4) || (stack && !aligned(stack, 4)) || (peak && !aligned(peak, 4)) ||
        (curvature && !aligned(curvature, 4)))
        return fail(KM_E_INVALID, "km_cig_moveout: misaligned pointer");
    if (curvature && (!offsets || !aligned(offsets, 4)))
        return fail(KM_E_INVALID, "km_cig_moveout: offsets NULL/misaligned with curvature requested");
    if (km::cig_lds_bytes(grid->n_bins, grid->nz, max_lag) > static_cast<size_t>(kMaxLds))
        return fail(KM_E_UNSUPPORTED, "km_cig_moveout: %d bins x %d depths do not fit in LDS", grid->n_bins,
                    grid->nz);
    if (grid->nx == 0 || grid->ny == 0) return KM_OK;
    {
        const km_status ist = injected("moveout launch");
        if (ist != KM_OK) return ist;
    }
    const hipError_t e = km::launch_cig(image, grid->n_bins, grid->ny, grid->nx, grid->nz, max_lag, z_lo, z_hi,
                                        offsets, stack, shift, peak, curvature, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? KM_OK : hip_fail(e, "moveout launch");
}

int32_t km_tile_count(int32_t op) { return (op == 0 || op == 1) ? shape_count(op) : 0; }

int32_t km_tile_levels(int32_t op) { return (op == 0 || op == 1) ? level_count(op) : 0; }

km_status km_tile_describe(int32_t op, int32_t tile, km_tile_info* out) {
    if (op != 0 && op != 1) return fail(KM_E_INVALID, "km_tile_describe: op must be 0 or 1");
    int shape = 0, level = 0;
    if (!decode_tile(op, tile, &shape, &level)) return fail(KM_E_INVALID, "km_tile_describe: tile out of range");
    if (!out) return fail(KM_E_INVALID, "km_tile_describe: out is NULL");
    const km::TileShape& S = op == 0 ? km::migrate_shape(shape) : km::demigrate_shape(shape);
    out->waves = S.waves;
    out->column_groups = S.column_groups;
    out->depth_slots = S.depth_slots;
    out->lds_budget = op == 0 ? static_cast<int>(std::min<double>(kMaxLds, S.lds_budget * kMigrateBudgetScale[level]))
                              : S.lds_budget;
    out->trace_quads = op == 0 ? 0 : (level > 0 ? level : S.max_quads);
    out->shape = shape;
    out->level = level;
    out->lds16 = op == 0 ? kMigrateLds16[level] : 0;
    return KM_OK;
}

int32_t km_tune_lookup(int32_t op, int32_t dtype, int32_t kind, int32_t time_precision, int32_t nz,
                       int32_t n_samples) {
    const TuneKey key = tune_key(op, dtype, kind, time_precision, nz, n_samples);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(key);
    return it == g_tune.end() ? -1 : it->second.tile;
}

km_status km_tune_record(int32_t op, int32_t dtype, int32_t kind, int32_t time_precision, int32_t nz,
                         int32_t n_samples, int32_t tile, float ms) {
    if (op != 0 && op != 1) return fail(KM_E_INVALID, "km_tune_record: op must be 0 or 1");
    if (kind < KIND_DSR || kind > KIND_LTABLE) return fail(KM_E_INVALID, "km_tune_record: unknown kind %d", kind);
    int shape = 0, level = 0;
    if (!decode_tile(op, tile, &shape, &level)) return fail(KM_E_INVALID, "km_tune_record: tile out of range");
    if (!tile_applies(op, tile, dtype, kind, time_precision))
        return fail(KM_E_INVALID, "km_tune_record: tile %d stages 16-bit traces, which this class does not have", tile);
    const TuneKey key = tune_key(op, dtype, kind, time_precision, nz, n_samples);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    g_tune[key] = TuneEntry{tile, ms};
    tune_save_locked();
    return KM_OK;
}

// km_tune and km_tune_ltable: lat (with table) selects the laterally varying tables.
static km_status tune_impl(int32_t op, const km_traces* traces, const km_grid* grid, const km_traveltime* tt,
                           const km_weight* weight, const km_ttable* table, const km_antialias* aa, const Lateral* lat,
                           float* image, int32_t reps, void* stream, int32_t* best_tile, float* best_ms) {
    if (op != 0 && op != 1) return fail(KM_E_INVALID, "km_tune: op must be 0 or 1");
    if (reps < 1) return fail(KM_E_INVALID, "km_tune: reps < 1");
    if (table && aa) return fail(KM_E_INVALID, "km_tune: table traveltimes and the anti-alias filter exclude each other");
    km_status st = check_traces(traces, true, "km_tune");
    if (st != KM_OK) return st;
    km_traveltime ttab_tt{};
    km_weight unit{KM_W_UNIT};
    if (table && !lat) {
        st = check_table(table, grid, "km_tune");
        if (st != KM_OK) return st;
    }
    if (table) {
        ttab_tt = km_traveltime{table->r2, table->r2, table->r2, table->time_precision};
        tt = &ttab_tt;
        weight = &unit;
    }
    if (aa) {
        st = check_antialias(aa, "km_tune");
        if (st == KM_OK) st = check_antialias_tt(tt, "km_tune");
        if (st != KM_OK) return st;
    }
    st = check_grid(grid, tt, weight, "km_tune");
    if (st != KM_OK) return st;
    if (op == 1 && traces->dtype != KM_F32) return fail(KM_E_UNSUPPORTED, "km_tune: demigrate output must be KM_F32");
    if (grid_empty(grid) || traces->n_traces == 0) return fail(KM_E_INVALID, "km_tune: empty problem");
    if (!image) return fail(KM_E_INVALID, "km_tune: image is NULL");
    const int kind = lat ? KIND_LTABLE : table ? KIND_TABLE : aa ? KIND_AA : KIND_DSR;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    hipError_t he = hipEventCreate(&e0);
    if (he != hipSuccess) return hip_fail(he, "hipEventCreate");
    he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        hipEventDestroy(e0);
        return hip_fail(he, "hipEventCreate");
    }
    int best = -1;
    float best_t = 0.0f;
    st = KM_OK;
    // every compiled shape at every variant level that applies to it
    for (int sh = 0; sh < shape_count(op) && st == KM_OK; ++sh) {
        for (int lv = 0; lv < level_count(op) && st == KM_OK; ++lv) {
            int d_shape = 0, d_level = 0;
            const int tile = sh + kTileLevelStride * lv;
            if (!decode_tile(op, tile, &d_shape, &d_level)) continue;
            km::Params P = base_params(traces, grid, tt, weight, image, 0);
            if (aa) {
                P.aa_max = aa->max_half;
                P.lt = (traces->n_samples + 2 * (2 * aa->max_half + 5) + 3) / 4 * 4;
            }
            if (table) P.ttab = table->t;
            if (shape_params(op, tile, P) != KM_OK) continue;
            if (op == 1 && lv > 0 && P.tb < 4 * lv) continue;  // the level's quads do not fit: same as a lower one
            st = run_op(op, traces, grid, tt, weight, image, 0, tile, s, table, aa, lat);
            if (st != KM_OK) break;
            hipEventRecord(e0, s);
            for (int r = 0; r < reps && st == KM_OK; ++r)
                st = run_op(op, traces, grid, tt, weight, image, 0, tile, s, table, aa, lat);
            hipEventRecord(e1, s);
            he = hipEventSynchronize(e1);
            if (he != hipSuccess) {
                st = hip_fail(he, "km_tune synchronise");
                break;
            }
            float ms = 0.0f;
            hipEventElapsedTime(&ms, e0, e1);
            ms /= reps;
            if (best < 0 || ms < best_t) {
                best = tile;
                best_t = ms;
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != KM_OK) return st;
    if (best < 0) return fail(KM_E_UNSUPPORTED, "km_tune: no tile fits this problem");
    st = km_tune_record(op, traces->dtype, kind, tt->time_precision, grid->nz, traces->n_samples, best, best_t);
    if (st != KM_OK) return st;
    if (best_tile) *best_tile = best;
    if (best_ms) *best_ms = best_t;
    return KM_OK;
}

km_status km_tune(int32_t op, const km_traces* traces, const km_grid* grid, const km_traveltime* tt,
                  const km_weight* weight, const km_ttable* table, const km_antialias* aa, float* image,
                  int32_t reps, void* stream, int32_t* best_tile, float* best_ms) {
    return tune_impl(op, traces, grid, tt, weight, table, aa, nullptr, image, reps, stream, best_tile, best_ms);
}

km_status km_tune_ltable(int32_t op, const km_traces* traces, const km_grid* grid, const km_ltable* ltab,
                         float* image, int32_t reps, void* stream, int32_t* best_tile, float* best_ms) {
    km_ttable tab;
    Lateral lat;
    const km_status st = check_ltable(ltab, grid, "km_tune_ltable", &tab, &lat);
    if (st != KM_OK) return st;
    const km_traveltime tt{tab.r2, tab.r2, tab.r2, tab.time_precision};
    const km_weight w{KM_W_UNIT};
    return tune_impl(op, traces, grid, &tt, &w, &tab, nullptr, &lat, image, reps, stream, best_tile, best_ms);
}

// ---- batched persistent migration -----------------------------------------

}  // extern "C"

namespace {

// A batched migration: the shape and kernel flags every problem shares, the
// problems' launch parameters and their work items, longest first.
struct BatchPlan {
    int tile = 0, shape = 0, has_tf = 0, weight = 0, prec = 0;
    std::vector<km::Params> P;
    std::vector<int4> items;  // (problem, bin, column tile or -1 - tile when empty, depth chunk)
    size_t lds = 0;
    int64_t max_slots = 0;    // largest per-problem item count (the cost buffer's length)
    int64_t n_slots = 0;      // items over all problems
};

km_status batch_plan(const km_problem* probs, int32_t n, int32_t tile, const char* who, BatchPlan& B) {
    if (!probs || n < 1) return fail(KM_E_INVALID, "%s: need n >= 1 problems", who);
    for (int i = 0; i < n; ++i) {
        km_status st = check_traces(&probs[i].traces, true, who);
        if (st != KM_OK) return st;
        st = check_grid(&probs[i].grid, &probs[i].tt, &probs[i].weight, who);
        if (st != KM_OK) return st;
        if (grid_empty(&probs[i].grid)) return fail(KM_E_INVALID, "%s: problem %d has an empty grid", who, i);
        if (!probs[i].image || !aligned(probs[i].image, 4))
            return fail(KM_E_INVALID, "%s: problem %d image NULL/misaligned", who, i);
        if ((probs[i].traces.t_first != 0.0) != (probs[0].traces.t_first != 0.0) ||
            probs[i].weight.kind != probs[0].weight.kind || probs[i].tt.time_precision != probs[0].tt.time_precision)
            return fail(KM_E_UNSUPPORTED,
                        "%s: all problems must share the weight kind, the time precision and t_first == 0 or not",
                        who);
    }
    int max_nz = 0, max_nt = 0;
    for (int i = 0; i < n; ++i) {
        max_nz = std::max(max_nz, probs[i].grid.nz);
        max_nt = std::max(max_nt, probs[i].traces.n_samples);
    }
    km_status st = pick_tile(0, tile, probs[0].traces.dtype, KIND_DSR, probs[0].tt.time_precision, max_nz, max_nt,
                             &B.tile);
    if (st != KM_OK) return st;
    B.shape = B.tile % kTileLevelStride;
    {
        // the batched kernels stage floats: a tuned 16-bit staging tile becomes
        // its float-staging level, a requested one is refused
        const int lv = B.tile / kTileLevelStride;
        if (kMigrateLds16[lv]) {
            if (tile >= 0) return fail(KM_E_UNSUPPORTED, "%s: 16-bit staging tiles are not batched", who);
            B.tile = B.shape + kTileLevelStride * kMigrateFloatLevel[lv];
        }
    }
    const km::TileShape& S = km::migrate_shape(B.shape);
    B.has_tf = probs[0].traces.t_first != 0.0 ? 1 : 0;
    B.weight = probs[0].weight.kind;
    B.prec = probs[0].tt.time_precision == KM_TIME_EXTENDED ? 1 : 0;
    B.P.resize(n);
    for (int i = 0; i < n; ++i) {
        km::Params& P = B.P[i];
        P = base_params(&probs[i].traces, &probs[i].grid, &probs[i].tt, &probs[i].weight, probs[i].image, 0);
        st = shape_params(0, B.tile, P);
        if (st != KM_OK) return st;
        if (P.n_traces > INT32_MAX)
            return fail(KM_E_UNSUPPORTED, "%s: problem %d has more than 2^31 - 1 traces", who, i);
        B.lds = std::max(B.lds, km::lds_bytes(P, S.depth_slots));
        const int64_t nslot = static_cast<int64_t>(P.n_bins) * P.n_zchunks * P.n_coltiles;
        if (nslot > (int64_t(1) << 31)) return fail(KM_E_UNSUPPORTED, "%s: problem %d has too many work items", who, i);
        B.max_slots = std::max(B.max_slots, nslot);
        B.n_slots += nslot;
    }
    return KM_OK;
}

// Work-item costs (pairs in aperture) from the counting kernel, written to
// d_costs (device, >= B.max_slots entries) one problem at a time and read
// back; the items are then ordered longest first.  Synchronises s.
km_status batch_items(BatchPlan& B, unsigned long long* d_costs, hipStream_t s, const char* who) {
    const km::TileShape& S = km::migrate_shape(B.shape);
    struct Item {
        unsigned long long cost;
        int4 w;
    };
    std::vector<Item> items;
    items.reserve(static_cast<size_t>(B.n_slots));
    std::vector<unsigned long long> h(static_cast<size_t>(std::max<int64_t>(B.max_slots, 1)));
    for (size_t i = 0; i < B.P.size(); ++i) {
        const km::Params& P = B.P[i];
        const int64_t nslot = static_cast<int64_t>(P.n_bins) * P.n_zchunks * P.n_coltiles;
        hipError_t e = km::launch_item_costs(P, S.depth_slots, S.waves * S.column_groups * 4, d_costs, s);
        if (e == hipSuccess && nslot > 0)
            e = hipMemcpyAsync(h.data(), d_costs, sizeof(unsigned long long) * nslot, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, who);
        for (int b = 0; b < P.n_bins; ++b)
            for (int zc = 0; zc < P.n_zchunks; ++zc)
                for (int tl = 0; tl < P.n_coltiles; ++tl) {
                    const unsigned long long c = h[(static_cast<int64_t>(b) * P.n_zchunks + zc) * P.n_coltiles + tl];
                    items.push_back({c, make_int4(static_cast<int>(i), b, c ? tl : -1 - tl, zc)});
                }
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.cost > b.cost; });
    B.items.resize(items.size());
    for (size_t k = 0; k < items.size(); ++k) B.items[k] = items[k].w;
    return KM_OK;
}

// Persistent grid: as many workgroups as can be resident at once.
km_status batch_grid(const BatchPlan& B, int device, int* n_wg, int* per_cu_out, const char* who) {
    const km::TileShape& S = km::migrate_shape(B.shape);
    const void* kfn = km::migrate_batch_kernel_ptr(B.shape, B.has_tf, B.weight, B.prec);
    if (B.lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 static_cast<int>(B.lds));
        if (e != hipSuccess) return hip_fail(e, who);
    }
    int per_cu = 0, n_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, S.waves * 64, B.lds);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return hip_fail(e, who);
    const int64_t n_items = static_cast<int64_t>(B.items.size());
    *n_wg = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(static_cast<int64_t>(std::max(per_cu, 1)) * n_cu,
                                                                      std::max<int64_t>(n_items, 1))));
    if (per_cu_out) *per_cu_out = per_cu;
    return KM_OK;
}

// Scratch of the allocation-free batched migration: one array per GPU (each
// device holds its own copy from module load to process end), laid out as
// [queue counter | problem table | work items, or the cost counts while
// they are measured].
constexpr size_t kScratchBytes = size_t(8) << 20;
constexpr size_t kScratchProblems = 4096;
constexpr size_t kScratchItemsOffset = 256 + kScratchProblems * sizeof(km::Params);
static_assert(kScratchItemsOffset % 256 == 0, "items start on a 256-byte boundary");
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch (looked up once per device, with the
// device current).  In host code the array's name is not a device address.
km_status scratch_ptr(int device, unsigned char** out) {
    if (device < 0 || device >= kMaxDevices) return fail(KM_E_UNSUPPORTED, "device %d: no scratch slot", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        g_scratch_ptr[device] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
    return KM_OK;
}

}  // namespace

extern "C" {

struct km_batch {
    int device = 0;
    BatchPlan plan;
    km::Params* d_probs = nullptr;
    int4* d_items = nullptr;
    unsigned int* d_counter = nullptr;
    int n_wg = 0;
    int per_cu = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static void batch_free(km_batch* b) {
    if (!b) return;
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    if (b->d_probs) hipFree(b->d_probs);
    if (b->d_items) hipFree(b->d_items);
    if (b->d_counter) hipFree(b->d_counter);
    delete b;
}

km_status km_batch_create(const km_problem* probs, int32_t n, int32_t op, int32_t tile, void* stream,
                          km_batch** out) {
    if (!out) return fail(KM_E_INVALID, "km_batch_create: out is NULL");
    *out = nullptr;
    if (op != 0 && op != 1) return fail(KM_E_INVALID, "km_batch_create: op must be 0 (migrate) or 1 (demigrate)");
    if (op == 1) return fail(KM_E_UNSUPPORTED, "km_batch_create: batched demigration is not built");
    hipStream_t s = static_cast<hipStream_t>(stream);
    km_batch* B = new (std::nothrow) km_batch();
    if (!B) return fail(KM_E_NOMEM, "km_batch_create: host allocation failed");
    hipGetDevice(&B->device);
    km_status st = batch_plan(probs, n, tile, "km_batch_create", B->plan);
    if (st != KM_OK) {
        batch_free(B);
        return st;
    }
    BatchPlan& L = B->plan;
    unsigned long long* d_costs = nullptr;
    hipError_t e = hipMalloc(&d_costs, sizeof(unsigned long long) * std::max<int64_t>(L.max_slots, 1));
    if (e != hipSuccess) {
        batch_free(B);
        return fail(KM_E_NOMEM, "km_batch_create: hipMalloc costs: %s", hipGetErrorString(e));
    }
    st = batch_items(L, d_costs, s, "km_batch_create: cost estimate");
    hipFree(d_costs);
    if (st != KM_OK) {
        batch_free(B);
        return st;
    }
    e = hipMalloc(&B->d_probs, sizeof(km::Params) * n);
    if (e == hipSuccess) e = hipMalloc(&B->d_items, sizeof(int4) * std::max<size_t>(L.items.size(), 1));
    if (e == hipSuccess) e = hipMalloc(&B->d_counter, sizeof(unsigned int));
    if (e != hipSuccess) {
        batch_free(B);
        return fail(KM_E_NOMEM, "km_batch_create: hipMalloc: %s", hipGetErrorString(e));
    }
    e = hipMemcpyAsync(B->d_probs, L.P.data(), sizeof(km::Params) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !L.items.empty())
        e = hipMemcpyAsync(B->d_items, L.items.data(), sizeof(int4) * L.items.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        batch_free(B);
        return hip_fail(e, "km_batch_create: upload");
    }
    st = batch_grid(L, B->device, &B->n_wg, &B->per_cu, "km_batch_create: occupancy");
    if (st != KM_OK) {
        batch_free(B);
        return st;
    }

    // Capture [queue reset, persistent kernel] once.
    hipStream_t cap = nullptr;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e1 = km::launch_reset_counter(B->d_counter, cap);
        hipError_t e2 = e1 == hipSuccess
                            ? km::launch_migrate_batch(L.shape, B->d_probs, B->d_items,
                                                       static_cast<int64_t>(L.items.size()), B->d_counter, L.has_tf,
                                                       L.weight, L.prec, B->n_wg, L.lds, cap)
                            : e1;
        e = hipStreamEndCapture(cap, &B->graph);
        if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
    if (cap) hipStreamDestroy(cap);
    if (e != hipSuccess) {
        batch_free(B);
        return hip_fail(e, "km_batch_create: graph capture");
    }
    *out = B;
    return KM_OK;
}

km_status km_batch_migrate_static(const km_problem* probs, int32_t n, int32_t tile, void* stream) {
    const char* who = "km_batch_migrate_static";
    hipStream_t s = static_cast<hipStream_t>(stream);
    BatchPlan L;
    km_status st = batch_plan(probs, n, tile, who, L);
    if (st != KM_OK) return st;
    if (static_cast<size_t>(n) > kScratchProblems)
        return fail(KM_E_UNSUPPORTED, "%s: %d problems exceed the static scratch's %zu", who, n, kScratchProblems);
    const size_t item_bytes = std::max(sizeof(int4) * static_cast<size_t>(L.n_slots),
                                       sizeof(unsigned long long) * static_cast<size_t>(L.max_slots));
    if (kScratchItemsOffset + item_bytes > kScratchBytes)
        return fail(KM_E_UNSUPPORTED, "%s: %lld work items need %zu bytes of scratch, more than the %zu available", who,
                    static_cast<long long>(L.n_slots), kScratchItemsOffset + item_bytes, kScratchBytes);
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    unsigned char* base = nullptr;
    st = scratch_ptr(device, &base);
    if (st != KM_OK) return st;
    auto* d_counter = reinterpret_cast<unsigned int*>(base);
    auto* d_probs = reinterpret_cast<km::Params*>(base + 256);
    auto* d_items = reinterpret_cast<int4*>(base + kScratchItemsOffset);
    auto* d_costs = reinterpret_cast<unsigned long long*>(base + kScratchItemsOffset);
    st = batch_items(L, d_costs, s, who);
    if (st != KM_OK) return st;
    e = hipMemcpyAsync(d_probs, L.P.data(), sizeof(km::Params) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !L.items.empty())
        e = hipMemcpyAsync(d_items, L.items.data(), sizeof(int4) * L.items.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host tables are released on return
    if (e != hipSuccess) return hip_fail(e, who);
    int n_wg = 0;
    st = batch_grid(L, device, &n_wg, nullptr, who);
    if (st != KM_OK) return st;
    st = injected("km_batch_migrate_static launch");
    if (st != KM_OK) return st;
    e = km::launch_reset_counter(d_counter, s);
    if (e == hipSuccess)
        e = km::launch_migrate_batch(L.shape, d_probs, d_items, static_cast<int64_t>(L.items.size()), d_counter,
                                     L.has_tf, L.weight, L.prec, n_wg, L.lds, s);
    return e == hipSuccess ? KM_OK : hip_fail(e, "km_batch_migrate_static launch");
}

km_status km_batch_run(km_batch* batch, void* stream) {
    if (!batch) return fail(KM_E_INVALID, "km_batch_run: batch is NULL");
    const km_status st = injected("km_batch_run launch");
    if (st != KM_OK) return st;
    const hipError_t e = hipGraphLaunch(batch->exec, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? KM_OK : hip_fail(e, "hipGraphLaunch");
}

km_status km_batch_info(const km_batch* batch, int64_t* n_items, int32_t* n_workgroups) {
    if (!batch) return fail(KM_E_INVALID, "km_batch_info: batch is NULL");
    if (n_items) *n_items = static_cast<int64_t>(batch->plan.items.size());
    if (n_workgroups) *n_workgroups = batch->n_wg;
    return KM_OK;
}

km_status km_batch_destroy(km_batch* batch) {
    if (!batch) return KM_OK;
    const hipError_t e = hipDeviceSynchronize();
    batch_free(batch);
    return e == hipSuccess ? KM_OK : hip_fail(e, "km_batch_destroy synchronise");
}

km_status km_probe_issue(int32_t kind, int32_t n_waves, int32_t iters, void* stream, float* ms) {
    if (kind < 0 || kind > 2 || n_waves < 1 || iters < 1 || !ms) return fail(KM_E_INVALID, "km_probe_issue: bad args");
    hipStream_t s = static_cast<hipStream_t>(stream);
    float* sink = nullptr;
    hipError_t e = hipMalloc(&sink, 256 * sizeof(float));
    if (e != hipSuccess) return hip_fail(e, "km_probe_issue hipMalloc");
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    e = km::launch_probe(kind, n_waves, iters, sink, s);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(a, s);
    if (e == hipSuccess) e = km::launch_probe(kind, n_waves, iters, sink, s);
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    hipEventDestroy(a);
    hipEventDestroy(b);
    hipFree(sink);
    if (e != hipSuccess) return hip_fail(e, "km_probe_issue");
    *ms = t;
    return KM_OK;
}

}  // extern "C"

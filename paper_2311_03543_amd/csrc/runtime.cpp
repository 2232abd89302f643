// libcompar host runtime: interface/variant registry, selection by runtime
// context, performance history, timing, verify mode and the built-in "gemm"
// variants.  Plays the part COMPAR gives to its generated glue code plus the
// StarPU runtime (Sec. 2.2): variants are registered at run time instead of
// being declared by pragmas, and the runtime picks one per call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <thread>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/compar.h"
#include "kernels.h"

#define CMP_API extern "C" __attribute__((visibility("default")))

namespace {

constexpr const char* kVersion = "compar-mi355x 0.1.0";
constexpr const char* kGemm = "gemm";
constexpr int kNumBuiltin = 4;
constexpr double kTolClasses[3] = {1e-5, 1e-3, 1e-2};

struct Param {
    std::string name;
    int type = 0, ndim = 0, mode = 0;
    std::string extent[4];
    bool operator==(const Param& o) const {
        if (name != o.name || type != o.type || ndim != o.ndim || mode != o.mode) return false;
        for (int i = 0; i < ndim; ++i)
            if (extent[i] != o.extent[i]) return false;
        return true;
    }
};

enum BuiltinKind { kNone = -1, kF32Simt = 0, kBf16x3 = 1, kFp8r = 2, kBf16 = 3 };

struct Variant {
    std::string name;
    int target = CMP_TARGET_HIP;
    cmp_variant_fn fn = nullptr;
    cmp_ws_fn ws = nullptr;
    double bound = 0;
    void* user = nullptr;
    uint64_t calls = 0;
};

struct Interface {
    std::string name;
    std::vector<Param> params;
    std::vector<Variant> variants;
    uint64_t mask = ~0ull;
    int forced = -1;
};

struct HistRow {
    int64_t M, N, K;
    int id, reps;
    float med, mn, mean;
};

// The history grouped by shape (first-appearance order): per shape the
// recorded median of each variant (NaN when missing) and the nearest-
// neighbour features (log2 M, log2 N, log2 K).
struct ShapeTable {
    std::vector<std::tuple<int64_t, int64_t, int64_t>> shapes;
    std::vector<std::vector<double>> med;
    std::vector<std::array<double, 3>> lg;
};

struct CacheKey {
    int64_t M, N, K;
    double tol;
    bool operator==(const CacheKey& o) const {
        return M == o.M && N == o.N && K == o.K && tol == o.tol;
    }
};
// A cached decision: the chosen id and the selector's predicted ln(us) for it
// (NaN when the selector predicts no time: the static choice).
struct CacheVal {
    int id;
    double pred_ln_us;
};
struct CacheHash {
    size_t operator()(const CacheKey& k) const {
        uint64_t h = 1469598103934665603ull;
        auto mix = [&](uint64_t v) { h = (h ^ v) * 1099511628211ull; };
        mix((uint64_t)k.M);
        mix((uint64_t)k.N);
        mix((uint64_t)k.K);
        uint64_t t;
        std::memcpy(&t, &k.tol, 8);
        mix(t);
        return (size_t)h;
    }
};

// splitmix64 (Steele, Lea and Flood 2014): output j of a generator seeded
// with `seed` is mix(seed + (j + 1) * golden).
inline uint64_t splitmix64_at(uint64_t seed, uint64_t j) {
    uint64_t z = seed + (j + 1) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
inline double u01(uint64_t z) { return (double)(z >> 11) * (1.0 / 9007199254740992.0); }

}  // namespace

// ---------------------------------------------------------------------------
// Fixed device workspace of cmp_gemm_variant_static: one array in the device
// code, which each GPU the library runs on holds until the process ends.  In
// host code its name is only a stand-in, never a device address:
// static_ws_address() asks the runtime, once per device and with that device
// current, for the address of this device's copy, and callers pass that.
namespace {
constexpr size_t kStaticWsBytes = CMP_STATIC_WS_BYTES;
__device__ __align__(256) uint8_t scratch[kStaticWsBytes];
constexpr int kMaxDevices = 64;
struct StaticWs {
    std::once_flag once;
    void* ptr = nullptr;
    hipError_t err = hipSuccess;
};
StaticWs g_static_ws[kMaxDevices];

// `device` must be the current device.
void* static_ws_address(int device, hipError_t* err) {
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    StaticWs& w = g_static_ws[device];
    std::call_once(w.once, [&w]() {
        void* p = nullptr;
        w.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        w.ptr = w.err == hipSuccess ? p : nullptr;
        if (w.err != hipSuccess) (void)hipGetLastError();
    });
    *err = w.err;
    return w.ptr;
}
}  // namespace

struct cmp_ctx {
    int device = -1;
    bool gpu = false;
    hipDeviceProp_t props{};
    std::vector<Interface> ifaces;
    std::string last_error;
    int selector = CMP_SEL_NN;
    uint32_t flags = 0;
    int split_k = 0;                  // 0: cost model; n >= 1: forced slice count
    std::vector<HistRow> history;
    uint64_t hist_gen = 0;            // bumped on every change of `history`
    // per-K-block workgroup time of each image kind on this device, derived
    // from the history (0: none yet, the built-in constant applies)
    mutable double step_ns[4] = {0, 0, 0, 0};
    mutable uint64_t step_gen = ~0ull;
    // shape table of the history, rebuilt when hist_gen or the variant count moves
    mutable ShapeTable shape_cache;
    mutable uint64_t shape_cache_gen = ~0ull;
    mutable size_t shape_cache_nvar = 0;
    std::unordered_map<CacheKey, CacheVal, CacheHash> cache;
    // learned selector
    std::vector<float> mlp_params;
    float mu_x[4] = {0, 0, 0, 0}, sd_x[4] = {1, 1, 1, 1};
    float mu_y[4] = {0, 0, 0, 0}, sd_y[4] = {1, 1, 1, 1};
    bool mlp_ready = false;
    // device memory owned by the library
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_pinned = false;  // cmp_reserve: never reallocate the workspace
    void* vws = nullptr;     // verify-mode workspace (C0 copy, probe vector, partial sums)
    void* static_ws = nullptr;              // this device's copy of the fixed array
    hipError_t static_ws_err = hipSuccess;  // why static_ws is null
    void* hbuf = nullptr;    // pinned host staging of the host variant (A | B | C)
    size_t hbuf_bytes = 0;
    size_t vws_bytes = 0;
    float* mlp_dev = nullptr;  // params | m | v | X | Y | loss | grad | infer io
    hipStream_t side = nullptr;
    // verify mode and fault injection
    double last_verify = -1.0;
    int fallbacks = 0;
    uint64_t verify_calls = 0;
    std::string fault_name;
    uint64_t fault_every = 0;
    // per-kernel timing of the built-in variants (HIP events around each launch)
    bool ktime = false;
    struct KEv {
        std::string name;
        hipEvent_t a, b;
    };
    std::vector<KEv> kpending;
    std::vector<hipEvent_t> kpool;
    std::map<std::string, std::pair<long long, double>> kstats;  // launches, total ms
    // per-call log (CMP_FLAG_LOG): one JSON line per cmp_gemm, written once the
    // call's HIP event pair has completed (records stay in call order)
    struct LogRec {
        uint64_t call;
        int64_t M, N, K;
        double tol;
        const char* how;         // how the variant was chosen
        int id;
        std::string name;
        double pred_us;          // NaN: no prediction
        double residual;         // NaN: no probe
        int fallbacks;           // fallbacks taken by this call
        hipEvent_t a, b;         // GPU variants: events around the variant's work
        double host_us;          // host variants: steady-clock duration
    };
    std::vector<LogRec> log_pending;
    FILE* log_fp = nullptr;      // nullptr: stderr
    uint64_t log_calls = 0;
    // COMPAR_VARIANTS / COMPAR_FORCE, applied by name to gemm variants as they register
    bool env_restrict = false;
    std::vector<std::string> env_allow;
    std::string env_force;
};

namespace {

int fail(cmp_ctx* c, int st, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->last_error = buf;
    }
    return st;
}

int hip_fail(cmp_ctx* c, hipError_t e, const char* what) {
    return fail(c, CMP_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                   \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return hip_fail(ctx, _e, #expr); \
    } while (0)

// Optional per-kernel timing: a scope that records a HIP event pair on the
// launch stream around one kernel launch of a built-in variant.
hipEvent_t kev_get(cmp_ctx* c) {
    if (!c->kpool.empty()) {
        hipEvent_t e = c->kpool.back();
        c->kpool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
struct KTimer {
    cmp_ctx* c;
    hipStream_t s;
    const char* name;
    hipEvent_t a = nullptr;
    KTimer(cmp_ctx* c_, hipStream_t s_, const char* n) : c(c_), s(s_), name(n) {
        if (c && c->ktime && (a = kev_get(c))) (void)hipEventRecord(a, s);
    }
    ~KTimer() {
        if (!a) return;
        hipEvent_t b = kev_get(c);
        if (!b) {
            c->kpool.push_back(a);
            return;
        }
        (void)hipEventRecord(b, s);
        c->kpending.push_back({name, a, b});
    }
};

// ---------------------------------------------------------------------------
// Per-call log (CMP_FLAG_LOG)

void json_str(std::string& out, const std::string& v) {
    out += '"';
    for (unsigned char ch : v) {
        if (ch == '"' || ch == '\\') {
            out += '\\';
            out += (char)ch;
        } else if (ch < 0x20) {
            char b[8];
            std::snprintf(b, sizeof b, "\\u%04x", ch);
            out += b;
        } else {
            out += (char)ch;
        }
    }
    out += '"';
}
void json_num(std::string& out, double v) {
    char b[32];
    if (std::isfinite(v)) std::snprintf(b, sizeof b, "%.9g", v);
    else std::snprintf(b, sizeof b, "null");
    out += b;
}
void log_write(cmp_ctx* c, const cmp_ctx::LogRec& r, double measured_us) {
    std::string l;
    char b[160];
    std::snprintf(b, sizeof b, "{\"call\": %llu, \"M\": %lld, \"N\": %lld, \"K\": %lld, \"tol\": ",
                  (unsigned long long)r.call, (long long)r.M, (long long)r.N, (long long)r.K);
    l += b;
    json_num(l, r.tol);
    l += ", \"selector\": \"";
    l += r.how;
    l += "\", \"variant\": ";
    json_str(l, r.name);
    std::snprintf(b, sizeof b, ", \"id\": %d, \"predicted_us\": ", r.id);
    l += b;
    json_num(l, r.pred_us);
    l += ", \"measured_us\": ";
    json_num(l, measured_us);
    l += ", \"residual\": ";
    json_num(l, r.residual);
    std::snprintf(b, sizeof b, ", \"fallbacks\": %d}\n", r.fallbacks);
    l += b;
    FILE* fp = c->log_fp ? c->log_fp : stderr;
    std::fwrite(l.data(), 1, l.size(), fp);
    std::fflush(fp);
}
// Write the pending records whose events have completed, in call order
// (stopping at the first one still running); with `wait`, all of them.
void log_drain(cmp_ctx* c, bool wait) {
    size_t done = 0;
    for (; done < c->log_pending.size(); ++done) {
        auto& r = c->log_pending[done];
        double us = r.host_us;
        if (r.b) {
            const hipError_t e = wait ? hipEventSynchronize(r.b) : hipEventQuery(r.b);
            if (e == hipErrorNotReady) break;
            float ms = 0.f;
            if (e == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                us = 1e3 * (double)ms;
            } else {
                us = NAN;
                (void)hipGetLastError();
            }
            c->kpool.push_back(r.a);
            c->kpool.push_back(r.b);
        }
        log_write(c, r, us);
    }
    c->log_pending.erase(c->log_pending.begin(), c->log_pending.begin() + (std::ptrdiff_t)done);
}

Interface* find_iface(cmp_ctx* c, const char* name) {
    if (!name) return nullptr;
    for (auto& f : c->ifaces)
        if (f.name == name) return &f;
    return nullptr;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ---------------------------------------------------------------------------
// Built-in gemm variants.  `user` is the context.

size_t ws_none(const void*, void*) { return 0; }

// Split-K count for the MFMA variants: the context's CU count decides when
// the output tiles alone leave CUs idle.
int cu_count(const void* user) {
    auto c = (const cmp_ctx*)user;
    return c && c->gpu && c->props.multiProcessorCount > 0 ? c->props.multiProcessorCount : 256;
}
constexpr int kMaxForcedSplits = 64;
int gemm_splits(const cmp_gemm_args* a, int64_t Kp_bytes, double step_ns, const void* user) {
    auto c = (const cmp_ctx*)user;
    const int nkb = (int)(Kp_bytes / cmp::kKBlockBytes);
    if (c && c->split_k > 0) {
        const int s = std::min(c->split_k, nkb);
        const int kbs = (nkb + s - 1) / s;
        return (nkb + kbs - 1) / kbs;      // every slice non-empty
    }
    return cmp::splits_for(a->M, a->N, nkb, step_ns, cu_count(user));
}
// partial sums of a split-K launch: splits x M x N floats, after the operand images
size_t partial_bytes(const cmp_gemm_args* a, int splits) {
    return splits > 1 ? (size_t)splits * a->M * a->N * sizeof(float) : 0;
}

// Operand images of the pre-passed (MFMA) variants.  Each keeps its images at
// the front of its workspace in a fixed order, which is also the order
// cmp_prepass_layout reports, followed by the split-K partial sums:
//   bf16   : A hi | B^T hi                                   (bf16 panel images)
//   bf16x3 : A hi | B^T hi | A lo | B^T lo                   (bf16 panel images)
//   fp8r   : A q | A r | B^T q | B^T r | E8M0 tile scales of A q, A r, B^T q, B^T r
//   fp6x3  : A hi | A lo | B^T hi | B^T lo | A scales | B^T scales (MX FP6 images)
// Mp and Np round M and N up to the 256-row MFMA tile; Kp rounds K up to 64
// (bf16, FP6) or 128 (FP8: whole 128 x 128 scale tiles).  Padding is zero.
enum ImageKind { kImgNone = -1, kImgBf16 = 0, kImgBf16x3 = 1, kImgFp8r = 2, kImgFp6x3 = 3 };
struct Images {
    int64_t Mp = 0, Np = 0, Kp = 0;
    int n = 0;
    size_t off[8] = {}, bytes[8] = {};
    size_t total = 0;  // bytes of all images (the split-K partials follow)
    uint8_t* at(void* base, int i) const { return (uint8_t*)base + off[i]; }
};
Images images_of(int kind, int64_t M, int64_t N, int64_t K) {
    Images I;
    I.Mp = round_up(std::max<int64_t>(M, 1), cmp::kMfmaTileM);
    I.Np = round_up(std::max<int64_t>(N, 1), cmp::kMfmaTileN);
    std::vector<size_t> b;
    if (kind == kImgBf16 || kind == kImgBf16x3) {
        I.Kp = round_up(std::max<int64_t>(K, 1), cmp::kBf16TileK);
        const size_t ab = (size_t)I.Mp * I.Kp * 2, bb = (size_t)I.Np * I.Kp * 2;
        b = {ab, bb};
        if (kind == kImgBf16x3) b.insert(b.end(), {ab, bb});
    } else if (kind == kImgFp8r) {
        I.Kp = round_up(std::max<int64_t>(K, 1), cmp::kFp8TileK);
        const size_t ab = (size_t)I.Mp * I.Kp, bb = (size_t)I.Np * I.Kp;
        const size_t as = (size_t)round_up((I.Mp / 128) * (I.Kp / 128), 256);
        const size_t bs = (size_t)round_up((I.Np / 128) * (I.Kp / 128), 256);
        b = {ab, ab, bb, bb, as, as, bs, bs};
    } else {
        I.Kp = round_up(std::max<int64_t>(K, 1), 64);
        const size_t nkb = (size_t)(I.Kp / 64);
        const size_t ac = (size_t)(I.Mp / 256) * nkb * cmp::kMx6CodeBlockBytes;
        const size_t bc = (size_t)(I.Np / 256) * nkb * cmp::kMx6CodeBlockBytes;
        const size_t as = (size_t)(I.Mp / 256) * nkb * cmp::kMx6ScaleBlockBytes;
        const size_t bs = (size_t)(I.Np / 256) * nkb * cmp::kMx6ScaleBlockBytes;
        b = {ac, ac, bc, bc, as, bs};
    }
    size_t o = 0;
    for (size_t i = 0; i < b.size(); ++i) {
        I.off[i] = o;
        I.bytes[i] = b[i];
        o += b[i];
    }
    I.n = (int)b.size();
    I.total = o;
    return I;
}
int image_kind(const Variant& v);

// Per-K-block time of one workgroup of an image variant on this device (ns),
// the price the split-K cost model puts on a K block.  Boards of one product
// differ by several percent in the clock their power limit allows, so it is
// taken from this context's own history where possible: over the timed shapes
// of the variant whose tiles fill every CU (no split) and whose K spans at
// least 64 blocks, (median time - the operand pre-pass at 5 TB/s) / (tile
// waves x K blocks), the median over those shapes, kept within [0.75, 1.33]
// of the constant measured at 8192^3.  Without such a shape, the constant.
double step_time(const cmp_ctx* c, int kind) {
    static constexpr double kConst[4] = {cmp::kStepNsBf16, cmp::kStepNsBf16x3, cmp::kStepNsFp8r,
                                         cmp::kStepNsFp6x3};
    if (!c || kind < 0 || kind > 3) return kind >= 0 && kind <= 3 ? kConst[kind] : cmp::kStepNsBf16;
    if (c->step_gen != c->hist_gen) {
        const Interface* f = nullptr;
        for (const auto& i : c->ifaces)
            if (i.name == kGemm) f = &i;
        const int cus = c->gpu && c->props.multiProcessorCount > 0 ? c->props.multiProcessorCount : 256;
        std::vector<double> per[4];
        for (const HistRow& r : c->history) {
            if (!f || r.id < 0 || r.id >= (int)f->variants.size() || !(r.med > 0)) continue;
            const int k = image_kind(f->variants[r.id]);
            if (k < 0) continue;
            const Images I = images_of(k, r.M, r.N, r.K);
            const int64_t nkb = (k == kImgBf16 || k == kImgBf16x3 ? I.Kp * 2 : I.Kp) / cmp::kKBlockBytes;
            const int64_t tiles = (I.Mp / cmp::kMfmaTileM) * (I.Np / cmp::kMfmaTileN);
            if (tiles < cus || nkb < 64) continue;
            const double waves = (double)((tiles + cus - 1) / cus);
            const double prepass_ns = (4.0 * (double)(r.M * r.K + r.K * r.N) + (double)I.total) / 5000.0;
            const double t = (double)r.med * 1e6 - prepass_ns;
            if (t > 0) per[k].push_back(t / (waves * (double)nkb));
        }
        for (int k = 0; k < 4; ++k) {
            double v = 0;
            if (!per[k].empty()) {
                std::sort(per[k].begin(), per[k].end());
                v = per[k][per[k].size() / 2];
                v = std::min(std::max(v, 0.75 * kConst[k]), 1.33 * kConst[k]);
            }
            c->step_ns[k] = v;
        }
        c->step_gen = c->hist_gen;
    }
    return c->step_ns[kind] > 0 ? c->step_ns[kind] : kConst[kind];
}

// Split-K count of an image variant: K blocks of 64 bytes (bf16: 32 values,
// FP8: 64 values, FP6: one 64-value block) priced at the variant's time per
// K block on this device.
int image_splits(int kind, const cmp_gemm_args* a, const Images& I, const void* user) {
    const double step = step_time((const cmp_ctx*)user, kind);
    return gemm_splits(a, kind == kImgBf16 || kind == kImgBf16x3 ? I.Kp * 2 : I.Kp, step, user);
}
size_t ws_images(int kind, const void* args, const void* user) {
    auto a = (const cmp_gemm_args*)args;
    const Images I = images_of(kind, a->M, a->N, a->K);
    return I.total + partial_bytes(a, image_splits(kind, a, I, user));
}
size_t ws_bf16(const void* args, void* user) { return ws_images(kImgBf16, args, user); }
size_t ws_bf16x3(const void* args, void* user) { return ws_images(kImgBf16x3, args, user); }
size_t ws_fp8r(const void* args, void* user) { return ws_images(kImgFp8r, args, user); }
size_t ws_fp6x3(const void* args, void* user) { return ws_images(kImgFp6x3, args, user); }

// Degenerate shapes shared by every built-in: nothing to do, or C = beta * C.
bool gemm_trivial(const cmp_gemm_args* a, hipStream_t s, int* st) {
    if (a->M == 0 || a->N == 0) {
        *st = CMP_OK;
        return true;
    }
    if (a->alpha == 0.f || a->K == 0) {
        *st = cmp::launch_scale_c(a->M, a->N, a->beta, a->C, a->ldc, s) == hipSuccess ? CMP_OK
                                                                                      : CMP_EHIP;
        return true;
    }
    return false;
}

int v_f32_simt(const void* args, void*, size_t, void* stream, void* user) {
    auto a = (const cmp_gemm_args*)args;
    auto s = (hipStream_t)stream;
    int st;
    if (gemm_trivial(a, s, &st)) return st;
    KTimer kt((cmp_ctx*)user, s, "gemm_f32_simt");
    return cmp::launch_gemm_f32_simt(a->M, a->N, a->K, a->alpha, a->A, a->lda, a->B, a->ldb,
                                     a->beta, a->C, a->ldc, s) == hipSuccess
               ? CMP_OK
               : CMP_EHIP;
}


// Sum of the split-K partials into C (nothing to do without a split).
int finish_split(cmp_ctx* c, const cmp_gemm_args* a, int splits, const float* partial,
                 hipStream_t s) {
    if (splits < 2) return CMP_OK;
    KTimer kt(c, s, "splitk_reduce");
    return cmp::launch_splitk_reduce(a->M, a->N, splits, partial, a->alpha, a->beta, a->C, a->ldc, s) ==
                   hipSuccess
               ? CMP_OK
               : CMP_EHIP;
}

// The pre-pass of an image variant: one kernel on the caller's stream that
// turns A and B into the variant's images at `base` (laid out by images_of),
// its workgroups interleaving the two operands (each alone leaves HBM
// bandwidth unused, and one launch saves a kernel boundary).
int prepass(cmp_ctx* c, int kind, const cmp_gemm_args* a, const Images& I, void* base,
            hipStream_t s) {
    // every pre-pass handles both operands in one launch, their workgroups interleaved
    if (kind == kImgBf16 || kind == kImgBf16x3) {
        const bool lo = kind == kImgBf16x3;
        KTimer kt(c, s, lo ? "split_bf16_hilo_ab" : "split_bf16_ab");
        return cmp::launch_split_bf16_pair(a->M, a->N, a->K, a->A, a->lda, a->B, a->ldb, I.Mp, I.Np, I.Kp,
                                           (uint16_t*)I.at(base, 0), lo ? (uint16_t*)I.at(base, 2) : nullptr,
                                           (uint16_t*)I.at(base, 1), lo ? (uint16_t*)I.at(base, 3) : nullptr,
                                           s) == hipSuccess
                   ? CMP_OK
                   : CMP_EHIP;
    }
    if (kind == kImgFp8r) {
        KTimer kt(c, s, "quant_fp8_ab");
        return cmp::launch_quant_fp8_pair(a->M, a->N, a->K, a->A, a->lda, a->B, a->ldb, I.Mp, I.Np, I.Kp,
                                          I.at(base, 0), I.at(base, 4), I.at(base, 1), I.at(base, 5),
                                          I.at(base, 2), I.at(base, 6), I.at(base, 3), I.at(base, 7),
                                          s) == hipSuccess
                   ? CMP_OK
                   : CMP_EHIP;
    }
    KTimer kt(c, s, "quant_mx6_ab");
    return cmp::launch_quant_mx6_pair(a->M, a->N, a->K, a->A, a->lda, a->B, a->ldb, I.Mp, I.Np, I.Kp,
                                      I.at(base, 0), I.at(base, 1), I.at(base, 4), I.at(base, 2),
                                      I.at(base, 3), I.at(base, 5), s) == hipSuccess
               ? CMP_OK
               : CMP_EHIP;
}

// An image variant: pre-pass, then its GEMM kernel over the images (with
// split-K partials after the images when the cost model splits K).
int run_images(cmp_ctx* c, int kind, const cmp_gemm_args* a, void* ws, hipStream_t s) {
    int st;
    if (gemm_trivial(a, s, &st)) return st;
    const Images I = images_of(kind, a->M, a->N, a->K);
    const int splits = image_splits(kind, a, I, c);
    auto* partial = (float*)((uint8_t*)ws + I.total);
    if ((st = prepass(c, kind, a, I, ws, s))) return st;
    hipError_t e;
    if (kind == kImgBf16 || kind == kImgBf16x3) {
        const bool lo = kind == kImgBf16x3;
        KTimer kt(c, s, lo ? "gemm_bf16x3_tn" : "gemm_bf16_tn");
        e = cmp::launch_gemm_bf16_tn(a->M, a->N, I.Kp, lo ? 3 : 1, a->alpha, (uint16_t*)I.at(ws, 0),
                                     lo ? (uint16_t*)I.at(ws, 2) : nullptr, (uint16_t*)I.at(ws, 1),
                                     lo ? (uint16_t*)I.at(ws, 3) : nullptr, a->beta, a->C, a->ldc,
                                     splits, partial, s);
    } else if (kind == kImgFp8r) {
        KTimer kt(c, s, "gemm_fp8r_tn");
        e = cmp::launch_gemm_fp8r_tn(a->M, a->N, I.Kp, a->alpha, I.at(ws, 0), I.at(ws, 1), I.at(ws, 4),
                                     I.at(ws, 5), I.at(ws, 2), I.at(ws, 3), I.at(ws, 6), I.at(ws, 7),
                                     a->beta, a->C, a->ldc, splits, partial, s);
    } else {
        KTimer kt(c, s, "gemm_fp6x3_tn");
        e = cmp::launch_gemm_fp6x3_tn(a->M, a->N, I.Kp, a->alpha, I.at(ws, 0), I.at(ws, 1), I.at(ws, 4),
                                      I.at(ws, 2), I.at(ws, 3), I.at(ws, 5), a->beta, a->C, a->ldc,
                                      splits, partial, s);
    }
    if (e != hipSuccess) return CMP_EHIP;
    return finish_split(c, a, splits, partial, s);
}
int v_bf16(const void* args, void* ws, size_t, void* stream, void* user) {
    return run_images((cmp_ctx*)user, kImgBf16, (const cmp_gemm_args*)args, ws, (hipStream_t)stream);
}
int v_bf16x3(const void* args, void* ws, size_t, void* stream, void* user) {
    return run_images((cmp_ctx*)user, kImgBf16x3, (const cmp_gemm_args*)args, ws, (hipStream_t)stream);
}
int v_fp8r(const void* args, void* ws, size_t, void* stream, void* user) {
    return run_images((cmp_ctx*)user, kImgFp8r, (const cmp_gemm_args*)args, ws, (hipStream_t)stream);
}
int v_fp6x3(const void* args, void* ws, size_t, void* stream, void* user) {
    return run_images((cmp_ctx*)user, kImgFp6x3, (const cmp_gemm_args*)args, ws, (hipStream_t)stream);
}
// The image kind of a registered variant (kImgNone: no operand pre-pass).
int image_kind(const Variant& v) {
    if (v.fn == v_bf16) return kImgBf16;
    if (v.fn == v_bf16x3) return kImgBf16x3;
    if (v.fn == v_fp8r) return kImgFp8r;
    if (v.fn == v_fp6x3) return kImgFp6x3;
    return kImgNone;
}

// The optional host variant: FP32 GEMM on the CPU.  In a GPU context the
// operands are device memory: A, B (and C when beta != 0) are copied to host
// buffers after the work already queued on the stream, multiplied, and C is
// copied back before the call returns (the call is synchronous).  In a
// host-only context the pointers are host memory and are used in place.
int v_host_f32(const void* args, void*, size_t, void* stream, void* user) {
    auto* c = (cmp_ctx*)user;
    auto a = (const cmp_gemm_args*)args;
    const int threads = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 16u);
    if (a->M == 0 || a->N == 0) return CMP_OK;
    if (!c->gpu) {
        cmp::host_gemm_f32(a->M, a->N, a->K, a->alpha, a->A, a->lda, a->B, a->ldb, a->beta, a->C, a->ldc,
                           threads);
        return CMP_OK;
    }
    auto s = (hipStream_t)stream;
    int st;
    if (gemm_trivial(a, s, &st)) return st;
    // pinned staging, grown on demand: A (M x K) | B (K x N) | C (M x N), tight
    const size_t na = (size_t)a->M * a->K, nb = (size_t)a->K * a->N, nc = (size_t)a->M * a->N;
    const size_t need = (na + nb + nc) * sizeof(float);
    if (need > c->hbuf_bytes) {
        if (c->hbuf && hipStreamSynchronize(s) == hipSuccess) (void)hipHostFree(c->hbuf);
        c->hbuf = nullptr;
        c->hbuf_bytes = 0;
        if (hipHostMalloc(&c->hbuf, need, hipHostMallocDefault) != hipSuccess) {
            c->hbuf = nullptr;
            (void)hipGetLastError();
            return fail(c, CMP_ENOMEM, "pinned host staging of %zu bytes failed", need);
        }
        c->hbuf_bytes = need;
    }
    float* hA = (float*)c->hbuf;
    float* hB = hA + na;
    float* hC = hB + nb;
    const size_t f = sizeof(float);
    // one linear copy when the rows are tight, a pitched copy otherwise
    auto get = [&](float* dst, const float* src, int64_t rows, int64_t cols, int64_t ld) {
        return ld == cols ? hipMemcpyAsync(dst, src, (size_t)rows * cols * f, hipMemcpyDeviceToHost, s)
                          : hipMemcpy2DAsync(dst, cols * f, src, ld * f, cols * f, rows, hipMemcpyDeviceToHost, s);
    };
    if (get(hA, a->A, a->M, a->K, a->lda) || get(hB, a->B, a->K, a->N, a->ldb) ||
        (a->beta != 0.f && get(hC, a->C, a->M, a->N, a->ldc)) || hipStreamSynchronize(s))
        return CMP_EHIP;
    cmp::host_gemm_f32(a->M, a->N, a->K, a->alpha, hA, a->K, hB, a->N, a->beta, hC, a->N, threads);
    const hipError_t e = a->ldc == a->N
        ? hipMemcpyAsync(a->C, hC, nc * f, hipMemcpyHostToDevice, s)
        : hipMemcpy2DAsync(a->C, a->ldc * f, hC, a->N * f, a->N * f, a->M, hipMemcpyHostToDevice, s);
    if (e != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return CMP_EHIP;
    return CMP_OK;
}

// ---------------------------------------------------------------------------

int validate_params(cmp_ctx* c, int n, const cmp_param_desc* p, std::vector<Param>* out) {
    if (n < 0 || (n > 0 && !p)) return fail(c, CMP_EINVAL, "bad parameter list");
    std::vector<Param> v;
    for (int i = 0; i < n; ++i) {
        if (!p[i].name || !*p[i].name) return fail(c, CMP_EINVAL, "parameter %d has no name", i);
        if (p[i].ndim < 0 || p[i].ndim > 4)
            return fail(c, CMP_EINVAL, "parameter %s: ndim must be 0..4", p[i].name);
        if (p[i].type < CMP_F32 || p[i].type > CMP_I64)
            return fail(c, CMP_EINVAL, "parameter %s: unknown type", p[i].name);
        if (p[i].mode < CMP_READ || p[i].mode > CMP_READWRITE)
            return fail(c, CMP_EINVAL, "parameter %s: unknown access mode", p[i].name);
        Param q;
        q.name = p[i].name;
        q.type = p[i].type;
        q.ndim = p[i].ndim;
        q.mode = p[i].mode;
        for (int d = 0; d < q.ndim; ++d) {
            if (!p[i].extent[d] || !*p[i].extent[d])
                return fail(c, CMP_EINVAL, "parameter %s: missing extent %d", p[i].name, d);
            q.extent[d] = p[i].extent[d];
        }
        for (auto& o : v)
            if (o.name == q.name) return fail(c, CMP_EDUP, "duplicate parameter %s", q.name.c_str());
        v.push_back(q);
    }
    // every extent is a literal or names a scalar parameter of the interface
    for (auto& q : v)
        for (int d = 0; d < q.ndim; ++d) {
            const std::string& e = q.extent[d];
            bool lit = std::all_of(e.begin(), e.end(), [](char ch) { return ch >= '0' && ch <= '9'; });
            if (lit) continue;
            bool found = false;
            for (auto& o : v)
                if (o.name == e && o.ndim == 0) found = true;
            if (!found)
                return fail(c, CMP_EINVAL, "parameter %s: extent %s names no scalar parameter",
                            q.name.c_str(), e.c_str());
        }
    *out = std::move(v);
    return CMP_OK;
}

int register_variant(cmp_ctx* c, const char* iface, const char* name, int target, int nparams,
                     const cmp_param_desc* params, cmp_variant_fn fn, cmp_ws_fn ws,
                     double bound, void* user, int* id_out);
void apply_env_to_variant(cmp_ctx* c, Interface* f, int id);

void register_builtins(cmp_ctx* c) {
    static const cmp_param_desc gemm_params[] = {
        {"M", CMP_I64, 0, {nullptr, nullptr, nullptr, nullptr}, CMP_READ},
        {"N", CMP_I64, 0, {nullptr, nullptr, nullptr, nullptr}, CMP_READ},
        {"K", CMP_I64, 0, {nullptr, nullptr, nullptr, nullptr}, CMP_READ},
        {"alpha", CMP_F32, 0, {nullptr, nullptr, nullptr, nullptr}, CMP_READ},
        {"beta", CMP_F32, 0, {nullptr, nullptr, nullptr, nullptr}, CMP_READ},
        {"A", CMP_F32, 2, {"M", "K", nullptr, nullptr}, CMP_READ},
        {"B", CMP_F32, 2, {"K", "N", nullptr, nullptr}, CMP_READ},
        {"C", CMP_F32, 2, {"M", "N", nullptr, nullptr}, CMP_READWRITE},
    };
    cmp_interface_declare(c, kGemm, 8, gemm_params);
    if (!c->gpu) return;
    int id;
    register_variant(c, kGemm, "f32_simt", CMP_TARGET_HIP, 0, nullptr, v_f32_simt, ws_none, 1e-5, c, &id);
    register_variant(c, kGemm, "bf16x3", CMP_TARGET_HIP, 0, nullptr, v_bf16x3, ws_bf16x3, 1e-5, c, &id);
    register_variant(c, kGemm, "fp8r", CMP_TARGET_HIP, 0, nullptr, v_fp8r, ws_fp8r, 1e-3, c, &id);
    register_variant(c, kGemm, "bf16", CMP_TARGET_HIP, 0, nullptr, v_bf16, ws_bf16, 1e-2, c, &id);
}

int register_variant(cmp_ctx* c, const char* iface, const char* name, int target, int nparams,
                     const cmp_param_desc* params, cmp_variant_fn fn, cmp_ws_fn ws,
                     double bound, void* user, int* id_out) {
    if (!iface || !name || !*name || !fn) return fail(c, CMP_EINVAL, "null interface, name or function");
    if (target != CMP_TARGET_HIP && target != CMP_TARGET_HOST)
        return fail(c, CMP_EINVAL, "unknown target %d", target);
    if (!(bound > 0) || !std::isfinite(bound)) return fail(c, CMP_EINVAL, "error bound must be > 0");
    if (target == CMP_TARGET_HIP && !c->gpu)
        return fail(c, CMP_EUNSUPPORTED, "HIP variant on a host-only context");
    Interface* f = find_iface(c, iface);
    if (params) {
        std::vector<Param> v;
        int st = validate_params(c, nparams, params, &v);
        if (st) return st;
        if (!f) {
            c->ifaces.push_back(Interface{});
            f = &c->ifaces.back();
            f->name = iface;
            f->params = std::move(v);
        } else if (!(f->params == v)) {
            return fail(c, CMP_ESIG, "variant %s: signature differs from interface %s", name, iface);
        }
    } else if (!f) {
        return fail(c, CMP_ENOTFOUND, "interface %s not declared and no parameters given", iface);
    }
    for (auto& v : f->variants)
        if (v.name == name) return fail(c, CMP_EDUP, "duplicate variant %s of %s", name, iface);
    if (f->variants.size() >= 64) return fail(c, CMP_EINVAL, "at most 64 variants per interface");
    Variant v;
    v.name = name;
    v.target = target;
    v.fn = fn;
    v.ws = ws;
    v.bound = bound;
    v.user = user;
    f->variants.push_back(v);
    const int id = (int)f->variants.size() - 1;
    apply_env_to_variant(c, f, id);
    if (id_out) *id_out = id;
    c->cache.clear();
    return CMP_OK;
}

// Resource restriction and forcing by name (the paper's STARPU_NCUDA /
// STARPU_NCPU runs, Sec. 3.2): read once at cmp_init, applied to every gemm
// variant when it registers.
void read_env(cmp_ctx* c) {
    if (const char* s = std::getenv("COMPAR_SELECTOR")) {
        std::string v = s;
        if (v == "static") c->selector = CMP_SEL_STATIC;
        else if (v == "nn") c->selector = CMP_SEL_NN;
        else if (v == "mlp") c->selector = CMP_SEL_MLP;
    }
    if (const char* s = std::getenv("COMPAR_VARIANTS")) {
        c->env_restrict = true;
        std::stringstream ss(s);
        std::string tok;
        while (std::getline(ss, tok, ','))
            if (!tok.empty()) c->env_allow.push_back(tok);
    }
    if (const char* s = std::getenv("COMPAR_FORCE")) c->env_force = s;
    if (const char* s = std::getenv("COMPAR_LOG")) {
        if (*s && (c->log_fp = std::fopen(s, "a"))) c->flags |= CMP_FLAG_LOG;
    }
    if (const char* s = std::getenv("COMPAR_FAULT")) {
        std::string v = s;
        auto p = v.find(':');
        if (p != std::string::npos) {
            c->fault_name = v.substr(0, p);
            c->fault_every = std::strtoull(v.c_str() + p + 1, nullptr, 10);
        }
    }
}

void apply_env_to_variant(cmp_ctx* c, Interface* f, int id) {
    if (f->name != kGemm) return;
    const std::string& n = f->variants[id].name;
    if (c->env_restrict &&
        std::find(c->env_allow.begin(), c->env_allow.end(), n) == c->env_allow.end())
        f->mask &= ~(1ull << id);
    if (!c->env_force.empty() && n == c->env_force) f->forced = id;
}

// ---------------------------------------------------------------------------
// Selection

double tie_key_bound(const Interface& f, int i) { return f.variants[i].bound; }

// argmin of t over the candidate ids; ties -> tighter bound, then lower id.
int argmin_tiebreak(const Interface& f, const std::vector<int>& cand, const std::vector<double>& t) {
    int best = -1;
    for (int i : cand) {
        if (!std::isfinite(t[i])) continue;
        if (best < 0 || std::make_tuple(t[i], tie_key_bound(f, i), i) <
                            std::make_tuple(t[best], tie_key_bound(f, best), best))
            best = i;
    }
    return best;
}

std::vector<int> admissible_ids(const Interface& f, double tol) {
    std::vector<int> v;
    for (size_t i = 0; i < f.variants.size(); ++i)
        if ((f.mask >> i & 1) && f.variants[i].bound <= tol) v.push_back((int)i);
    return v;
}

// Distinct shapes of the history in order of first appearance, with the last
// recorded median per variant (NaN where none).
ShapeTable shape_table(const cmp_ctx* c, size_t nvar) {
    ShapeTable T;
    std::map<std::tuple<int64_t, int64_t, int64_t>, size_t> idx;
    for (auto& r : c->history) {
        auto key = std::make_tuple(r.M, r.N, r.K);
        auto it = idx.find(key);
        size_t s;
        if (it == idx.end()) {
            s = T.shapes.size();
            idx[key] = s;
            T.shapes.push_back(key);
            T.med.emplace_back(nvar, NAN);
        } else {
            s = it->second;
        }
        if (r.id >= 0 && (size_t)r.id < nvar) T.med[s][r.id] = r.med;
    }
    T.lg.reserve(T.shapes.size());
    for (auto& sh : T.shapes)
        T.lg.push_back({std::log2((double)std::get<0>(sh)), std::log2((double)std::get<1>(sh)),
                        std::log2((double)std::get<2>(sh))});
    return T;
}
// The selectors read the table on every uncached decision; build it once per
// history change.
const ShapeTable& shapes_of(const cmp_ctx* c, size_t nvar) {
    if (c->shape_cache_gen != c->hist_gen || c->shape_cache_nvar != nvar) {
        c->shape_cache = shape_table(c, nvar);
        c->shape_cache_gen = c->hist_gen;
        c->shape_cache_nvar = nvar;
    }
    return c->shape_cache;
}

int select_static(const cmp_ctx* c, const Interface& f, const std::vector<int>& adm) {
    const ShapeTable& T = shapes_of(c, f.variants.size());
    std::vector<double> tot(f.variants.size(), 0.0);
    size_t used = 0;
    for (size_t s = 0; s < T.shapes.size(); ++s) {
        bool complete = true;
        for (int i : adm)
            if (!std::isfinite(T.med[s][i])) complete = false;
        if (!complete) continue;
        ++used;
        for (int i : adm) tot[i] += T.med[s][i];
    }
    if (used == 0) {
        std::vector<double> z(f.variants.size(), 0.0);
        return argmin_tiebreak(f, adm, z);
    }
    return argmin_tiebreak(f, adm, tot);
}

int select_nn(const cmp_ctx* c, const Interface& f, const std::vector<int>& adm, int64_t M,
              int64_t N, int64_t K) {
    const ShapeTable& T = shapes_of(c, f.variants.size());
    const double q0 = std::log2((double)M), q1 = std::log2((double)N), q2 = std::log2((double)K);
    int best = -1;
    double bd = 0;
    for (size_t s = 0; s < T.shapes.size(); ++s) {
        bool any = false;
        for (int i : adm)
            if (std::isfinite(T.med[s][i])) any = true;
        if (!any) continue;
        const double d0 = T.lg[s][0] - q0;
        const double d1 = T.lg[s][1] - q1;
        const double d2 = T.lg[s][2] - q2;
        const double d = d0 * d0 + d1 * d1 + d2 * d2;
        if (best < 0 || d < bd) {
            best = (int)s;
            bd = d;
        }
    }
    if (best < 0) return -1;
    return argmin_tiebreak(f, adm, T.med[best]);
}

// ln(microseconds) of variant i at the nearest history shape that timed it
// (log2-space distance, as select_nn); infinity when no shape did.
double nn_log_us(const cmp_ctx* c, const Interface& f, int i, int64_t M, int64_t N, int64_t K) {
    const ShapeTable& T = shapes_of(c, f.variants.size());
    const double q0 = std::log2((double)std::max<int64_t>(M, 1));
    const double q1 = std::log2((double)std::max<int64_t>(N, 1));
    const double q2 = std::log2((double)std::max<int64_t>(K, 1));
    int best = -1;
    double bd = 0;
    for (size_t s = 0; s < T.shapes.size(); ++s) {
        if (!std::isfinite(T.med[s][i])) continue;
        const double d0 = T.lg[s][0] - q0, d1 = T.lg[s][1] - q1, d2 = T.lg[s][2] - q2;
        const double d = d0 * d0 + d1 * d1 + d2 * d2;
        if (best < 0 || d < bd) {
            best = (int)s;
            bd = d;
        }
    }
    return best < 0 ? INFINITY : std::log(T.med[best][i] * 1000.0);
}

}  // namespace

int mlp_predict(cmp_ctx* c, int n, const float* Xraw, float* Yraw);

namespace {

int do_select_batch(cmp_ctx* c, Interface* f, int n, const cmp_context* q, int* ids) {
    std::vector<int> pending;
    for (int r = 0; r < n; ++r) {
        const cmp_context& x = q[r];
        if (x.M < 0 || x.N < 0 || x.K < 0) return fail(c, CMP_EINVAL, "negative dimension");
        if (!(x.tol > 0)) return fail(c, CMP_EINVAL, "tolerance must be > 0");
        if (x.dtype != CMP_F32) return fail(c, CMP_EUNSUPPORTED, "only CMP_F32 operands are supported");
        std::vector<int> adm = admissible_ids(*f, x.tol);
        if (adm.empty())
            return fail(c, CMP_ENOVARIANT, "no enabled variant meets tol %g", x.tol);
        if (f->forced >= 0) {
            if (std::find(adm.begin(), adm.end(), f->forced) == adm.end())
                return fail(c, CMP_ENOVARIANT, "forced variant %s does not meet tol %g",
                            f->variants[f->forced].name.c_str(), x.tol);
            ids[r] = f->forced;
            continue;
        }
        if (adm.size() == 1) {
            ids[r] = adm[0];
            continue;
        }
        auto it = c->cache.find(CacheKey{x.M, x.N, x.K, x.tol});
        if (it != c->cache.end()) {
            ids[r] = it->second.id;
            continue;
        }
        ids[r] = -1;
        pending.push_back(r);
    }
    if (pending.empty()) return CMP_OK;

    std::vector<float> pred;  // MLP predictions (ln us) for pending rows
    const bool use_mlp = c->selector == CMP_SEL_MLP && c->mlp_ready && f->name == kGemm && c->gpu;
    if (use_mlp) {
        std::vector<float> X(pending.size() * 4);
        for (size_t p = 0; p < pending.size(); ++p) {
            const cmp_context& x = q[pending[p]];
            X[4 * p + 0] = (float)std::log2((double)std::max<int64_t>(x.M, 1));
            X[4 * p + 1] = (float)std::log2((double)std::max<int64_t>(x.N, 1));
            X[4 * p + 2] = (float)std::log2((double)std::max<int64_t>(x.K, 1));
            X[4 * p + 3] = (float)std::log10(x.tol);
        }
        pred.resize(pending.size() * 4);
        int st = mlp_predict(c, (int)pending.size(), X.data(), pred.data());
        if (st) return st;
    }
    for (size_t p = 0; p < pending.size(); ++p) {
        const cmp_context& x = q[pending[p]];
        std::vector<int> adm = admissible_ids(*f, x.tol);
        int id = -1;
        double pred_ln = NAN;
        if (use_mlp) {
            // the network predicts ln(us) of the four default built-ins; any
            // other variant is estimated from the history's nearest shape
            std::vector<double> t(f->variants.size(), INFINITY);
            for (int i : adm)
                t[i] = i < kNumBuiltin ? pred[4 * p + i] : nn_log_us(c, *f, i, x.M, x.N, x.K);
            id = argmin_tiebreak(*f, adm, t);
            if (id >= 0) pred_ln = t[id];
        }
        if (id < 0 && c->selector != CMP_SEL_STATIC) {
            id = select_nn(c, *f, adm, x.M, x.N, x.K);
            if (id >= 0) pred_ln = nn_log_us(c, *f, id, x.M, x.N, x.K);
        }
        if (id < 0) id = select_static(c, *f, adm);
        if (id < 0) return fail(c, CMP_ENOVARIANT, "selection failed");
        ids[pending[p]] = id;
        c->cache[CacheKey{x.M, x.N, x.K, x.tol}] = CacheVal{id, pred_ln};
    }
    return CMP_OK;
}

// ---------------------------------------------------------------------------
// Workspace

int ensure_ws(cmp_ctx* c, size_t need) {
    if (need <= c->ws_bytes) return CMP_OK;
    if (c->ws_pinned)
        return fail(c, CMP_ENOMEM, "call needs %zu workspace bytes, %zu are reserved (cmp_reserve)", need,
                    c->ws_bytes);
    // in-flight work on any stream may still read the old buffer
    HIP_TRY(c, hipDeviceSynchronize());
    if (c->ws) HIP_TRY(c, hipFree(c->ws));
    c->ws = nullptr;
    c->ws_bytes = 0;
    size_t sz = std::max<size_t>(need + need / 4, 1 << 20);
    if (hipMalloc(&c->ws, sz) != hipSuccess) {
        c->ws = nullptr;
        (void)hipGetLastError();
        return fail(c, CMP_ENOMEM, "workspace allocation of %zu bytes failed", sz);
    }
    c->ws_bytes = sz;
    return CMP_OK;
}

int ensure_vws(cmp_ctx* c, size_t need) {
    if (need <= c->vws_bytes) return CMP_OK;
    HIP_TRY(c, hipDeviceSynchronize());
    if (c->vws) HIP_TRY(c, hipFree(c->vws));
    c->vws = nullptr;
    c->vws_bytes = 0;
    size_t sz = std::max<size_t>(need + need / 4, 1 << 16);
    if (hipMalloc(&c->vws, sz) != hipSuccess) {
        c->vws = nullptr;
        (void)hipGetLastError();
        return fail(c, CMP_ENOMEM, "verify workspace allocation of %zu bytes failed", sz);
    }
    c->vws_bytes = sz;
    return CMP_OK;
}

int check_gemm_args(cmp_ctx* c, const cmp_gemm_args* a) {
    if (!a) return fail(c, CMP_EINVAL, "null args");
    if (a->M < 0 || a->N < 0 || a->K < 0) return fail(c, CMP_EINVAL, "negative dimension");
    if (a->M == 0 || a->N == 0) return CMP_OK;
    if (!a->C) return fail(c, CMP_EINVAL, "null C");
    if (a->ldc < std::max<int64_t>(a->N, 1)) return fail(c, CMP_EINVAL, "ldc < N");
    if (a->alpha != 0.f && a->K > 0) {
        if (!a->A || !a->B) return fail(c, CMP_EINVAL, "null A or B");
        if (a->lda < std::max<int64_t>(a->K, 1)) return fail(c, CMP_EINVAL, "lda < K");
        if (a->ldb < std::max<int64_t>(a->N, 1)) return fail(c, CMP_EINVAL, "ldb < N");
    }
    if (a->M > (int64_t)1 << 31 || a->N > (int64_t)1 << 31 || a->K > (int64_t)1 << 31)
        return fail(c, CMP_EINVAL, "dimension above 2^31");
    return CMP_OK;
}

int run_variant(cmp_ctx* c, Interface& f, int id, const void* args, void* stream) {
    Variant& v = f.variants[id];
    ++v.calls;
    if (c->fault_every && v.name == c->fault_name && v.calls % c->fault_every == 0)
        return fail(c, CMP_EHIP, "injected fault in variant %s (call %llu)", v.name.c_str(),
                    (unsigned long long)v.calls);
    size_t need = v.ws ? v.ws(args, v.user) : 0;
    if (need && v.target == CMP_TARGET_HIP) {
        int st = ensure_ws(c, need);
        if (st) return st;
    }
    int st = v.fn(args, need ? c->ws : nullptr, need, stream, v.user);
    if (st != CMP_OK) {
        if (c->last_error.empty() || st == CMP_EHIP) {
            hipError_t e = hipGetLastError();
            return fail(c, st, "variant %s failed (%d): %s", v.name.c_str(), st,
                        e != hipSuccess ? hipGetErrorString(e) : "");
        }
        return st;
    }
    return CMP_OK;
}

double verify_threshold(double tol, int64_t M) {
    // one Rademacher probe: the estimate's relative spread is about 1/sqrt(2M);
    // allow four standard deviations before calling it a failure
    return tol * (1.0 + 4.0 / std::sqrt(2.0 * (double)std::max<int64_t>(M, 1)));
}

// Verify workspace: [y: K doubles | pad] [out: 2 doubles | pad] [x: N doubles]
// [old C: M x N floats, only when beta != 0]
struct VLayout {
    size_t out_d, x_d, c0_b, total_b;
};
VLayout vlayout(const cmp_gemm_args* a, bool keep_c0) {
    VLayout L;
    L.out_d = (size_t)round_up(a->K + 2, 32);
    L.x_d = L.out_d + 32;
    L.c0_b = (size_t)round_up((int64_t)((L.x_d + (size_t)a->N) * 8), 256);
    L.total_b = L.c0_b + (keep_c0 ? (size_t)a->M * (size_t)a->N * 4 : 0);
    return L;
}

// c0 (read only when beta != 0) has leading dimension ldc0: N for the packed
// copy verify mode keeps, the caller's ldc for cmp_freivalds.
int probe(cmp_ctx* c, const cmp_gemm_args* a, const float* c0, int64_t ldc0, const double* x_dev,
          hipStream_t s, double* est) {
    const VLayout L = vlayout(a, false);
    double* base = (double*)c->vws;  // sized by the caller (ensure_vws with vlayout)
    double* out = base + L.out_d;
    HIP_TRY(c, cmp::launch_freivalds(a->M, a->N, a->K, a->alpha, a->A, a->lda, a->B, a->ldb,
                                     a->beta, c0, ldc0, a->C, a->ldc, x_dev, base, out, s));
    double h[2];
    HIP_TRY(c, hipMemcpyAsync(h, out, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    *est = h[1] > 0 ? std::sqrt(h[0]) / std::sqrt(h[1]) : std::sqrt(h[0]);
    return CMP_OK;
}

// Re-select among `allowed` (a subset of the admissible ids) without touching
// the decision cache or the caller-visible mask / forced state.
int reselect(cmp_ctx* c, Interface* f, const cmp_context& q, const std::vector<int>& allowed,
             int* id) {
    uint64_t m = 0;
    for (int i : allowed) m |= 1ull << i;
    const uint64_t saved = f->mask;
    const int saved_forced = f->forced;
    auto cache = std::move(c->cache);
    c->cache.clear();
    f->mask = m;
    f->forced = -1;
    int st = do_select_batch(c, f, 1, &q, id);
    f->mask = saved;
    f->forced = saved_forced;
    c->cache = std::move(cache);
    return st;
}

}  // namespace

// ===========================================================================
// C ABI

CMP_API const char* cmp_version(void) { return kVersion; }

CMP_API const char* cmp_status_string(int s) {
    switch (s) {
        case CMP_OK: return "CMP_OK";
        case CMP_EINVAL: return "CMP_EINVAL";
        case CMP_EDUP: return "CMP_EDUP";
        case CMP_ESIG: return "CMP_ESIG";
        case CMP_ENOTFOUND: return "CMP_ENOTFOUND";
        case CMP_ENOVARIANT: return "CMP_ENOVARIANT";
        case CMP_EUNSUPPORTED: return "CMP_EUNSUPPORTED";
        case CMP_EHIP: return "CMP_EHIP";
        case CMP_ENOMEM: return "CMP_ENOMEM";
        case CMP_ECHECK: return "CMP_ECHECK";
        case CMP_ENODATA: return "CMP_ENODATA";
        default: return "unknown status";
    }
}

CMP_API int cmp_init(int device, cmp_ctx** out) {
    if (!out) return CMP_EINVAL;
    *out = nullptr;
    cmp_ctx* c = new (std::nothrow) cmp_ctx();
    if (!c) return CMP_ENOMEM;
    c->device = device;
    if (device >= 0) {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess || device >= n) {
            delete c;
            return CMP_EHIP;
        }
        if (hipSetDevice(device) != hipSuccess || hipGetDeviceProperties(&c->props, device) != hipSuccess) {
            delete c;
            return CMP_EHIP;
        }
        if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return CMP_EHIP;
        }
        c->gpu = true;
        c->static_ws = static_ws_address(device, &c->static_ws_err);
    }
    read_env(c);
    register_builtins(c);
    *out = c;
    return CMP_OK;
}

CMP_API int cmp_terminate(cmp_ctx* c) {
    if (!c) return CMP_OK;
    if (c->gpu) (void)hipSetDevice(c->device);
    log_drain(c, true);
    if (c->log_fp) std::fclose(c->log_fp);
    if (c->gpu) {
        (void)hipSetDevice(c->device);
        if (c->side) (void)hipStreamSynchronize(c->side);
        (void)hipDeviceSynchronize();
        if (c->ws) (void)hipFree(c->ws);
        if (c->vws) (void)hipFree(c->vws);
        if (c->hbuf) (void)hipHostFree(c->hbuf);
        if (c->mlp_dev) (void)hipFree(c->mlp_dev);
        for (auto& k : c->kpending) {
            (void)hipEventDestroy(k.a);
            (void)hipEventDestroy(k.b);
        }
        for (auto e : c->kpool) (void)hipEventDestroy(e);
        if (c->side) (void)hipStreamDestroy(c->side);
    }
    delete c;
    return CMP_OK;
}

CMP_API const char* cmp_last_error(const cmp_ctx* c) { return c ? c->last_error.c_str() : "null context"; }

CMP_API int cmp_device(const cmp_ctx* c, int* device, char* arch, size_t arch_len, int* cus,
                       int* clock_khz) {
    if (!c) return CMP_EINVAL;
    if (device) *device = c->device;
    if (arch && arch_len) {
        std::snprintf(arch, arch_len, "%s", c->gpu ? c->props.gcnArchName : "host");
    }
    if (cus) *cus = c->gpu ? c->props.multiProcessorCount : 0;
    if (clock_khz) *clock_khz = c->gpu ? c->props.clockRate : 0;
    return CMP_OK;
}

CMP_API int cmp_interface_declare(cmp_ctx* c, const char* iface, int n, const cmp_param_desc* p) {
    if (!c) return CMP_EINVAL;
    if (!iface || !*iface) return fail(c, CMP_EINVAL, "null interface name");
    if (find_iface(c, iface)) return fail(c, CMP_EDUP, "duplicate interface %s", iface);
    std::vector<Param> v;
    int st = validate_params(c, n, p, &v);
    if (st) return st;
    c->ifaces.push_back(Interface{});
    c->ifaces.back().name = iface;
    c->ifaces.back().params = std::move(v);
    return CMP_OK;
}

CMP_API int cmp_variant_register(cmp_ctx* c, const char* iface, const char* name, int target,
                                 int nparams, const cmp_param_desc* params, cmp_variant_fn fn,
                                 cmp_ws_fn ws, double bound, void* user, int* id_out) {
    if (!c) return CMP_EINVAL;
    return register_variant(c, iface, name, target, nparams, params, fn, ws, bound, user, id_out);
}

CMP_API int cmp_variant_count(cmp_ctx* c, const char* iface, int* n) {
    if (!c || !n) return CMP_EINVAL;
    Interface* f = find_iface(c, iface);
    if (!f) return fail(c, CMP_ENOTFOUND, "unknown interface");
    *n = (int)f->variants.size();
    return CMP_OK;
}

CMP_API int cmp_variant_info(cmp_ctx* c, const char* iface, int id, const char** name, int* target,
                             double* bound) {
    if (!c) return CMP_EINVAL;
    Interface* f = find_iface(c, iface);
    if (!f) return fail(c, CMP_ENOTFOUND, "unknown interface");
    if (id < 0 || id >= (int)f->variants.size()) return fail(c, CMP_EINVAL, "bad variant id %d", id);
    if (name) *name = f->variants[id].name.c_str();
    if (target) *target = f->variants[id].target;
    if (bound) *bound = f->variants[id].bound;
    return CMP_OK;
}

CMP_API int cmp_variant_find(cmp_ctx* c, const char* iface, const char* name, int* id) {
    if (!c || !name || !id) return CMP_EINVAL;
    Interface* f = find_iface(c, iface);
    if (!f) return fail(c, CMP_ENOTFOUND, "unknown interface");
    for (size_t i = 0; i < f->variants.size(); ++i)
        if (f->variants[i].name == name) {
            *id = (int)i;
            return CMP_OK;
        }
    return fail(c, CMP_ENOTFOUND, "no variant %s", name);
}

CMP_API int cmp_set_variant_mask(cmp_ctx* c, const char* iface, uint64_t mask) {
    if (!c) return CMP_EINVAL;
    Interface* f = find_iface(c, iface);
    if (!f) return fail(c, CMP_ENOTFOUND, "unknown interface");
    f->mask = mask;
    c->cache.clear();
    return CMP_OK;
}

CMP_API int cmp_force_variant(cmp_ctx* c, const char* iface, int id) {
    if (!c) return CMP_EINVAL;
    Interface* f = find_iface(c, iface);
    if (!f) return fail(c, CMP_ENOTFOUND, "unknown interface");
    if (id >= (int)f->variants.size()) return fail(c, CMP_EINVAL, "bad variant id %d", id);
    f->forced = id < 0 ? -1 : id;
    return CMP_OK;
}

CMP_API int cmp_selector_set(cmp_ctx* c, int kind) {
    if (!c) return CMP_EINVAL;
    if (kind < CMP_SEL_STATIC || kind > CMP_SEL_MLP) return fail(c, CMP_EINVAL, "unknown selector");
    c->selector = kind;
    c->cache.clear();
    return CMP_OK;
}

CMP_API int cmp_set_flags(cmp_ctx* c, uint32_t flags) {
    if (!c) return CMP_EINVAL;
    if (flags & ~(uint32_t)(CMP_FLAG_VERIFY | CMP_FLAG_LOG)) return fail(c, CMP_EINVAL, "unknown flag bits 0x%x", flags);
    c->flags = flags;
    return CMP_OK;
}

CMP_API int cmp_set_log_file(cmp_ctx* c, const char* path) {
    if (!c) return CMP_EINVAL;
    FILE* fp = nullptr;
    if (path && *path && !(fp = std::fopen(path, "a")))
        return fail(c, CMP_EINVAL, "cannot open log file %s", path);
    log_drain(c, true);   // earlier records go to the earlier sink
    if (c->log_fp) std::fclose(c->log_fp);
    c->log_fp = fp;
    return CMP_OK;
}

CMP_API int cmp_log_flush(cmp_ctx* c) {
    if (!c) return CMP_EINVAL;
    log_drain(c, true);
    return CMP_OK;
}

CMP_API int cmp_register_builtin(cmp_ctx* c, const char* name, int* id) {
    if (!c || !name) return CMP_EINVAL;
    int vid = -1, st;
    if (std::strcmp(name, "host_f32") == 0) {
        st = register_variant(c, kGemm, "host_f32", CMP_TARGET_HOST, 0, nullptr, v_host_f32, ws_none, 1e-5, c,
                              &vid);
    } else if (std::strcmp(name, "fp6x3") == 0) {
        if (!c->gpu) return fail(c, CMP_EUNSUPPORTED, "fp6x3 needs a GPU context");
        st = register_variant(c, kGemm, "fp6x3", CMP_TARGET_HIP, 0, nullptr, v_fp6x3, ws_fp6x3, 1e-2, c, &vid);
    } else {
        return fail(c, CMP_ENOTFOUND, "no optional built-in named %s", name);
    }
    if (st) return st;
    if (id) *id = vid;
    return CMP_OK;
}

CMP_API int cmp_set_split_k(cmp_ctx* c, int splits) {
    if (!c) return CMP_EINVAL;
    if (splits < 0 || splits > kMaxForcedSplits)
        return fail(c, CMP_EINVAL, "split count must be 0 (automatic) or 1..%d", kMaxForcedSplits);
    c->split_k = splits;
    return CMP_OK;
}

CMP_API int cmp_reserve(cmp_ctx* c, int64_t M, int64_t N, int64_t K) {
    if (!c) return CMP_EINVAL;
    if (M < 0 || N < 0 || K < 0) return fail(c, CMP_EINVAL, "negative dimension");
    if (!c->gpu) return fail(c, CMP_EUNSUPPORTED, "cmp_reserve needs a GPU context");
    if (M == 0 && N == 0 && K == 0) {
        c->ws_pinned = false;
        return CMP_OK;
    }
    Interface* f = find_iface(c, kGemm);
    cmp_gemm_args a{};
    a.M = std::max<int64_t>(M, 1);
    a.N = std::max<int64_t>(N, 1);
    a.K = std::max<int64_t>(K, 1);
    a.lda = a.K;
    a.ldb = a.ldc = a.N;
    size_t need = 0;
    for (size_t i = 0; i < f->variants.size(); ++i) {
        const Variant& v = f->variants[i];
        if ((f->mask >> i & 1) && v.target == CMP_TARGET_HIP && v.ws) need = std::max(need, v.ws(&a, v.user));
    }
    c->ws_pinned = false;
    const int st = need ? ensure_ws(c, need) : CMP_OK;
    if (st) return st;
    c->ws_pinned = true;
    return CMP_OK;
}

CMP_API int cmp_split_k(cmp_ctx* c, int id, int64_t M, int64_t N, int64_t K, int* splits) {
    if (!c || !splits || M < 0 || N < 0 || K < 0) return CMP_EINVAL;
    Interface* f = find_iface(c, kGemm);
    if (!f) return fail(c, CMP_ENOTFOUND, "unknown interface");
    if (id < 0 || id >= (int)f->variants.size()) return fail(c, CMP_EINVAL, "bad variant id %d", id);
    cmp_gemm_args a{};
    a.M = M;
    a.N = N;
    a.K = K;
    const int kind = image_kind(f->variants[id]);
    if (M == 0 || N == 0 || K == 0 || f->variants[id].user != c || kind == kImgNone)
        *splits = 1;
    else
        *splits = image_splits(kind, &a, images_of(kind, M, N, K), c);
    return CMP_OK;
}

CMP_API int cmp_admissible(cmp_ctx* c, const char* iface, const cmp_context* q, uint64_t* mask) {
    if (!c || !q || !mask) return CMP_EINVAL;
    Interface* f = find_iface(c, iface);
    if (!f) return fail(c, CMP_ENOTFOUND, "unknown interface");
    if (!(q->tol > 0)) return fail(c, CMP_EINVAL, "tolerance must be > 0");
    uint64_t m = 0;
    for (int i : admissible_ids(*f, q->tol)) m |= 1ull << i;
    *mask = m;
    return CMP_OK;
}

CMP_API int cmp_select(cmp_ctx* c, const char* iface, const cmp_context* q, int* id) {
    if (!c || !q || !id) return CMP_EINVAL;
    Interface* f = find_iface(c, iface);
    if (!f) return fail(c, CMP_ENOTFOUND, "unknown interface");
    return do_select_batch(c, f, 1, q, id);
}

CMP_API int cmp_select_batch(cmp_ctx* c, const char* iface, int n, const cmp_context* q, int* ids) {
    if (!c || n < 0 || (n > 0 && (!q || !ids))) return CMP_EINVAL;
    Interface* f = find_iface(c, iface);
    if (!f) return fail(c, CMP_ENOTFOUND, "unknown interface");
    return do_select_batch(c, f, n, q, ids);
}

CMP_API int cmp_gemm_variant(cmp_ctx* c, int id, const cmp_gemm_args* a, void* stream) {
    if (!c) return CMP_EINVAL;
    Interface* f = find_iface(c, kGemm);
    int st = check_gemm_args(c, a);
    if (st) return st;
    if (id < 0 || id >= (int)f->variants.size()) return fail(c, CMP_EINVAL, "bad variant id %d", id);
    if (f->variants[id].target == CMP_TARGET_HIP && !c->gpu)
        return fail(c, CMP_EUNSUPPORTED, "HIP variant on a host-only context");
    return run_variant(c, *f, id, a, stream);
}

CMP_API int cmp_gemm_variant_static(cmp_ctx* c, int id, const cmp_gemm_args* a, void* stream) {
    if (!c) return CMP_EINVAL;
    if (!c->gpu) return fail(c, CMP_EUNSUPPORTED, "the fixed workspace needs a GPU context");
    Interface* f = find_iface(c, kGemm);
    int st = check_gemm_args(c, a);
    if (st) return st;
    if (id < 0 || id >= (int)f->variants.size()) return fail(c, CMP_EINVAL, "bad variant id %d", id);
    Variant& v = f->variants[id];
    if (v.target != CMP_TARGET_HIP)
        return fail(c, CMP_EUNSUPPORTED, "variant %s does not run on the GPU", v.name.c_str());
    if (!c->static_ws)
        return fail(c, CMP_EHIP, "address of the fixed workspace unavailable: %s",
                    hipGetErrorString(c->static_ws_err));
    const size_t need = v.ws ? v.ws(a, v.user) : 0;
    if (need > kStaticWsBytes)
        return fail(c, CMP_ENOMEM, "variant %s needs %zu workspace bytes for %lld x %lld x %lld; the fixed "
                    "workspace holds %zu", v.name.c_str(), need, (long long)a->M, (long long)a->N,
                    (long long)a->K, kStaticWsBytes);
    const bool ktime = c->ktime;   // per-kernel timing creates events: off for this call
    c->ktime = false;
    ++v.calls;
    st = v.fn(a, need ? c->static_ws : nullptr, need, stream, v.user);
    c->ktime = ktime;
    if (st != CMP_OK) {
        if (c->last_error.empty() || st == CMP_EHIP) {
            hipError_t e = hipGetLastError();
            return fail(c, st, "variant %s failed (%d): %s", v.name.c_str(), st,
                        e != hipSuccess ? hipGetErrorString(e) : "");
        }
        return st;
    }
    return CMP_OK;
}

CMP_API int cmp_call_host(cmp_ctx* c, const char* iface, int id, const void* args) {
    if (!c) return CMP_EINVAL;
    Interface* f = find_iface(c, iface);
    if (!f) return fail(c, CMP_ENOTFOUND, "unknown interface");
    if (id < 0 || id >= (int)f->variants.size()) return fail(c, CMP_EINVAL, "bad variant id %d", id);
    if (f->variants[id].target != CMP_TARGET_HOST) return fail(c, CMP_EINVAL, "not a host variant");
    return run_variant(c, *f, id, args, nullptr);
}

CMP_API int cmp_gemm(cmp_ctx* c, const cmp_gemm_args* a, double tol, void* stream, int* chosen) {
    if (!c) return CMP_EINVAL;
    int st = check_gemm_args(c, a);
    if (st) return st;
    if (!(tol > 0)) return fail(c, CMP_EINVAL, "tolerance must be > 0");
    Interface* f = find_iface(c, kGemm);
    const cmp_context q{a->M, a->N, a->K, CMP_F32, tol};
    int id = -1;
    st = do_select_batch(c, f, 1, &q, &id);
    if (st) return st;
    const bool verify = (c->flags & CMP_FLAG_VERIFY) && c->gpu && a->M > 0 && a->N > 0;
    auto s = (hipStream_t)stream;
    // CMP_FLAG_LOG: HIP events around the run that produces C (none while the
    // stream is being captured: the record then has no measured time)
    const bool logging = (c->flags & CMP_FLAG_LOG) != 0;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    double host_us = NAN;
    bool capturing = false;
    const int fallbacks0 = c->fallbacks;
    struct EvGuard {   // events not handed to a log record go back to the pool
        cmp_ctx* c;
        hipEvent_t* a;
        hipEvent_t* b;
        ~EvGuard() {
            if (*a) c->kpool.push_back(*a);
            if (*b) c->kpool.push_back(*b);
        }
    } ev_guard{c, &ev_a, &ev_b};
    auto timed_run = [&](int vid) -> int {
        const bool hip_v = f->variants[vid].target == CMP_TARGET_HIP && c->gpu;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (logging && hip_v && hipStreamIsCapturing(s, &cs) == hipSuccess) {
            capturing = cs != hipStreamCaptureStatusNone;
            if (!capturing && !ev_a) ev_a = kev_get(c);
            if (!capturing && ev_a) (void)hipEventRecord(ev_a, s);
        }
        const auto t0 = std::chrono::steady_clock::now();
        const int rst = run_variant(c, *f, vid, a, stream);
        const auto t1 = std::chrono::steady_clock::now();
        host_us = hip_v ? NAN : std::chrono::duration<double, std::micro>(t1 - t0).count();
        if (logging && hip_v && ev_a && cs == hipStreamCaptureStatusNone) {
            if (!ev_b) ev_b = kev_get(c);
            if (ev_b) (void)hipEventRecord(ev_b, s);
        }
        return rst;
    };
    auto log_call = [&](int vid, double residual) {
        if (!logging) return;
        const char* how = c->selector == CMP_SEL_MLP ? "mlp" : (c->selector == CMP_SEL_NN ? "nn" : "static");
        double pred = NAN;
        const auto it = c->cache.find(CacheKey{a->M, a->N, a->K, tol});
        if (f->forced >= 0) how = "forced";
        else if (admissible_ids(*f, tol).size() == 1) how = "only";
        else if (it != c->cache.end() && it->second.id == vid) pred = std::exp(it->second.pred_ln_us);
        if (ev_a && !ev_b) {
            c->kpool.push_back(ev_a);
            ev_a = nullptr;
        }
        c->log_pending.push_back(cmp_ctx::LogRec{++c->log_calls, a->M, a->N, a->K, tol, how, vid,
                                                 f->variants[vid].name, pred, residual,
                                                 c->fallbacks - fallbacks0, ev_a, ev_b, host_us});
        ev_a = ev_b = nullptr;
        if (!capturing) log_drain(c, false);   // no event queries inside a capture
    };
    float* c0 = nullptr;
    double* xdev = nullptr;
    auto restore_c = [&]() -> int {
        if (c0)
            HIP_TRY(c, hipMemcpy2DAsync(a->C, (size_t)a->ldc * 4, c0, (size_t)a->N * 4,
                                        (size_t)a->N * 4, (size_t)a->M, hipMemcpyDeviceToDevice, s));
        return CMP_OK;
    };
    if (verify) {
        // keep the old C when beta != 0: the probe and a re-run both need it
        const VLayout L = vlayout(a, a->beta != 0.f);
        st = ensure_vws(c, L.total_b);
        if (st) return st;
        xdev = (double*)c->vws + L.x_d;
        if (a->beta != 0.f) {
            c0 = (float*)((char*)c->vws + L.c0_b);
            HIP_TRY(c, hipMemcpy2DAsync(c0, (size_t)a->N * 4, a->C, (size_t)a->ldc * 4,
                                        (size_t)a->N * 4, (size_t)a->M, hipMemcpyDeviceToDevice, s));
        }
        HIP_TRY(c, cmp::launch_rademacher(a->N, 0x5eedull + c->verify_calls++, xdev, s));
    }
    st = timed_run(id);
    if (st != CMP_OK && st != CMP_EINVAL) {
        // a failing variant gets one fallback: the best other admissible variant
        std::vector<int> rest;
        for (int i : admissible_ids(*f, tol))
            if (i != id) rest.push_back(i);
        if (rest.empty()) return st;
        int id2 = -1;
        if ((st = reselect(c, f, q, rest, &id2))) return st;
        ++c->fallbacks;
        if ((st = restore_c())) return st;
        if ((st = timed_run(id2))) return st;
        id = id2;
    }
    double residual = NAN;
    if (verify) {
        double est = 0;
        if ((st = probe(c, a, c0, a->N, xdev, s, &est))) return st;
        c->last_verify = est;
        if (est > verify_threshold(tol, a->M)) {
            // rerun once with the best admissible variant of strictly tighter bound
            const double b = f->variants[id].bound;
            std::vector<int> tighter;
            for (int i : admissible_ids(*f, tol))
                if (f->variants[i].bound < b) tighter.push_back(i);
            if (tighter.empty()) {
                log_call(id, est);
                return fail(c, CMP_ECHECK, "residual probe %.3g exceeds tol %g (variant %s)", est,
                            tol, f->variants[id].name.c_str());
            }
            int id2 = -1;
            if ((st = reselect(c, f, q, tighter, &id2))) return st;
            ++c->fallbacks;
            if ((st = restore_c())) return st;
            if ((st = timed_run(id2))) return st;
            id = id2;
            if ((st = probe(c, a, c0, a->N, xdev, s, &est))) return st;
            c->last_verify = est;
            if (est > verify_threshold(tol, a->M)) {
                log_call(id, est);
                return fail(c, CMP_ECHECK, "residual probe %.3g exceeds tol %g after fallback", est, tol);
            }
        }
        residual = est;
    }
    log_call(id, residual);
    if (chosen) *chosen = id;
    return CMP_OK;
}

CMP_API int cmp_gemm_stream(cmp_ctx* c, int n, const cmp_gemm_args* reqs, const double* tols,
                            const uint32_t* flags, int sync, void* stream, int* chosen, double* lat_us,
                            int* done) {
    if (done) *done = 0;
    if (!c) return CMP_EINVAL;
    if (n < 0 || (n > 0 && (!reqs || !tols))) return fail(c, CMP_EINVAL, "bad request list");
    const uint32_t saved = c->flags;
    auto s = (hipStream_t)stream;
    int st = CMP_OK;
    for (int i = 0; i < n; ++i) {
        if (flags) c->flags = (saved & ~(uint32_t)CMP_FLAG_VERIFY) | (flags[i] & (uint32_t)CMP_FLAG_VERIFY);
        const auto t0 = std::chrono::steady_clock::now();
        int id = -1;
        st = cmp_gemm(c, &reqs[i], tols[i], stream, &id);
        if (st == CMP_OK && sync && c->gpu) {
            const hipError_t e = hipStreamSynchronize(s);
            if (e != hipSuccess) st = hip_fail(c, e, "request stream");
        }
        if (st != CMP_OK) break;
        if (sync && lat_us)
            lat_us[i] = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
        if (chosen) chosen[i] = id;
        if (done) *done = i + 1;
    }
    c->flags = saved;
    return st;
}

CMP_API int cmp_time_variant(cmp_ctx* c, int id, const cmp_gemm_args* a, int warmup, int reps,
                             void* stream, float* med, float* mn, float* mean) {
    if (!c) return CMP_EINVAL;
    if (reps < 1 || warmup < 0) return fail(c, CMP_EINVAL, "reps must be >= 1");
    Interface* f = find_iface(c, kGemm);
    int st = check_gemm_args(c, a);
    if (st) return st;
    if (id < 0 || id >= (int)f->variants.size()) return fail(c, CMP_EINVAL, "bad variant id %d", id);
    const bool host = f->variants[id].target == CMP_TARGET_HOST;
    if (!host && !c->gpu) return fail(c, CMP_EUNSUPPORTED, "HIP variant on a host-only context");
    auto s = (hipStream_t)stream;
    for (int w = 0; w < warmup; ++w)
        if ((st = run_variant(c, *f, id, a, stream))) return st;
    std::vector<float> t(reps);
    if (host) {
        for (int r = 0; r < reps; ++r) {
            auto t0 = std::chrono::steady_clock::now();
            if ((st = run_variant(c, *f, id, a, stream))) return st;
            auto t1 = std::chrono::steady_clock::now();
            t[r] = std::chrono::duration<float, std::milli>(t1 - t0).count();
        }
    } else {
        std::vector<hipEvent_t> ev(2 * reps);
        for (auto& e : ev) HIP_TRY(c, hipEventCreate(&e));
        int rst = CMP_OK;
        for (int r = 0; r < reps && !rst; ++r) {
            (void)hipEventRecord(ev[2 * r], s);
            rst = run_variant(c, *f, id, a, stream);
            (void)hipEventRecord(ev[2 * r + 1], s);
        }
        hipError_t se = hipStreamSynchronize(s);
        for (int r = 0; r < reps && !rst && se == hipSuccess; ++r)
            (void)hipEventElapsedTime(&t[r], ev[2 * r], ev[2 * r + 1]);
        for (auto& e : ev) (void)hipEventDestroy(e);
        if (rst) return rst;
        if (se != hipSuccess) return hip_fail(c, se, "hipStreamSynchronize");
    }
    std::vector<float> srt = t;
    std::sort(srt.begin(), srt.end());
    const float m = (reps % 2) ? srt[reps / 2] : 0.5f * (srt[reps / 2 - 1] + srt[reps / 2]);
    double sum = 0;
    for (float v : t) sum += v;
    if (med) *med = m;
    if (mn) *mn = srt[0];
    if (mean) *mean = (float)(sum / reps);
    return CMP_OK;
}

CMP_API int cmp_history_add(cmp_ctx* c, int64_t M, int64_t N, int64_t K, int id, int reps, float med,
                            float mn, float mean) {
    if (!c) return CMP_EINVAL;
    Interface* f = find_iface(c, kGemm);
    if (M <= 0 || N <= 0 || K <= 0) return fail(c, CMP_EINVAL, "history shape must be positive");
    if (id < 0 || id >= (int)f->variants.size()) return fail(c, CMP_EINVAL, "bad variant id %d", id);
    if (!(med > 0) || !std::isfinite(med)) return fail(c, CMP_EINVAL, "median must be > 0");
    c->history.push_back(HistRow{M, N, K, id, reps, med, mn, mean});
    ++c->hist_gen;
    c->cache.clear();
    return CMP_OK;
}

CMP_API int cmp_calibrate(cmp_ctx* c, int nshapes, const int64_t* mnk, const float* A,
                          const float* B, float* C, int warmup, int reps, void* stream) {
    if (!c) return CMP_EINVAL;
    if (nshapes < 0 || (nshapes > 0 && !mnk)) return fail(c, CMP_EINVAL, "bad shape list");
    Interface* f = find_iface(c, kGemm);
    std::map<std::tuple<int64_t, int64_t, int64_t, int>, bool> have;
    for (auto& r : c->history) have[std::make_tuple(r.M, r.N, r.K, r.id)] = true;
    for (int s = 0; s < nshapes; ++s) {
        cmp_gemm_args a{};
        a.M = mnk[3 * s];
        a.N = mnk[3 * s + 1];
        a.K = mnk[3 * s + 2];
        a.lda = a.K;
        a.ldb = a.N;
        a.ldc = a.N;
        a.alpha = 1.f;
        a.beta = 0.f;
        a.A = A;
        a.B = B;
        a.C = C;
        if (a.M <= 0 || a.N <= 0 || a.K <= 0) return fail(c, CMP_EINVAL, "calibration shape must be positive");
        for (size_t v = 0; v < f->variants.size(); ++v) {
            if (!(f->mask >> v & 1)) continue;
            if (have.count(std::make_tuple(a.M, a.N, a.K, (int)v))) continue;
            float med, mn, mean;
            int st = cmp_time_variant(c, (int)v, &a, warmup, reps, stream, &med, &mn, &mean);
            if (st) return st;
            c->history.push_back(HistRow{a.M, a.N, a.K, (int)v, reps, med, mn, mean});
            ++c->hist_gen;
        }
    }
    c->cache.clear();
    return CMP_OK;
}

CMP_API int cmp_history_count(cmp_ctx* c, int* n) {
    if (!c || !n) return CMP_EINVAL;
    *n = (int)c->history.size();
    return CMP_OK;
}

CMP_API int cmp_history_get(cmp_ctx* c, int row, int64_t* mnk, int* id, int* reps, float* med,
                            float* mn, float* mean) {
    if (!c) return CMP_EINVAL;
    if (row < 0 || row >= (int)c->history.size()) return fail(c, CMP_EINVAL, "bad history row");
    const HistRow& r = c->history[row];
    if (mnk) {
        mnk[0] = r.M;
        mnk[1] = r.N;
        mnk[2] = r.K;
    }
    if (id) *id = r.id;
    if (reps) *reps = r.reps;
    if (med) *med = r.med;
    if (mn) *mn = r.mn;
    if (mean) *mean = r.mean;
    return CMP_OK;
}

CMP_API int cmp_history_clear(cmp_ctx* c) {
    if (!c) return CMP_EINVAL;
    c->history.clear();
    ++c->hist_gen;
    c->cache.clear();
    return CMP_OK;
}

namespace {
std::string device_signature(const cmp_ctx* c) {
    char buf[256];
    if (c->gpu)
        std::snprintf(buf, sizeof buf, "arch=%s cus=%d clock_khz=%d", c->props.gcnArchName,
                      c->props.multiProcessorCount, c->props.clockRate);
    else
        std::snprintf(buf, sizeof buf, "arch=host cus=0 clock_khz=0");
    return buf;
}
}  // namespace

CMP_API int cmp_history_save(cmp_ctx* c, const char* path) {
    if (!c || !path) return CMP_EINVAL;
    Interface* f = find_iface(c, kGemm);
    std::ofstream o(path);
    if (!o) return fail(c, CMP_EINVAL, "cannot open %s", path);
    o << "# compar-history v1\n";
    o << "# device " << device_signature(c) << "\n";
    o << "# lib " << kVersion << "\n";
    o << "# M N K variant reps median_ms min_ms mean_ms\n";
    char line[256];
    for (auto& r : c->history) {
        std::snprintf(line, sizeof line, "%lld %lld %lld %s %d %.9g %.9g %.9g\n", (long long)r.M,
                      (long long)r.N, (long long)r.K, f->variants[r.id].name.c_str(), r.reps, r.med,
                      r.mn, r.mean);
        o << line;
    }
    if (!o) return fail(c, CMP_EINVAL, "write to %s failed", path);
    return CMP_OK;
}

CMP_API int cmp_history_load(cmp_ctx* c, const char* path, int force) {
    if (!c || !path) return CMP_EINVAL;
    Interface* f = find_iface(c, kGemm);
    std::ifstream in(path);
    if (!in) return fail(c, CMP_EINVAL, "cannot open %s", path);
    std::string line;
    std::vector<HistRow> rows;
    bool header = false;
    while (std::getline(in, line)) {
        if (line.empty()) continue;
        if (line[0] == '#') {
            if (line.rfind("# compar-history v1", 0) == 0) header = true;
            if (line.rfind("# device ", 0) == 0 && !force) {
                std::string sig = line.substr(9);
                if (sig != device_signature(c))
                    return fail(c, CMP_EINVAL, "history recorded on '%s', this device is '%s'",
                                sig.c_str(), device_signature(c).c_str());
            }
            continue;
        }
        std::istringstream ss(line);
        long long M, N, K;
        std::string name;
        HistRow r{};
        if (!(ss >> M >> N >> K >> name >> r.reps >> r.med >> r.mn >> r.mean))
            return fail(c, CMP_EINVAL, "malformed history line: %s", line.c_str());
        // the same rules as cmp_history_add: positive shape, finite positive median
        if (M <= 0 || N <= 0 || K <= 0 || !(r.med > 0) || !std::isfinite(r.med))
            return fail(c, CMP_EINVAL, "invalid history line: %s", line.c_str());
        r.M = M;
        r.N = N;
        r.K = K;
        r.id = -1;
        for (size_t i = 0; i < f->variants.size(); ++i)
            if (f->variants[i].name == name) r.id = (int)i;
        if (r.id < 0) {
            if (force) continue;
            return fail(c, CMP_ENOTFOUND, "history names unknown variant %s", name.c_str());
        }
        rows.push_back(r);
    }
    if (!header) return fail(c, CMP_EINVAL, "%s is not a compar history file", path);
    c->history.insert(c->history.end(), rows.begin(), rows.end());
    ++c->hist_gen;
    c->cache.clear();
    return CMP_OK;
}

// ---------------------------------------------------------------------------
// Learned selector

namespace {

constexpr int kMlpP = cmp::kMlpParams;

// device block: params | m | v | X | Y | loss(steps) | grad | infer-out
struct MlpDev {
    float *params, *m, *v, *X, *Y, *grad, *part;
};

int mlp_dev(cmp_ctx* c, MlpDev* d) {
    if (!c->gpu) return fail(c, CMP_EUNSUPPORTED, "learned selector needs a GPU context");
    const size_t floats =
        3 * (size_t)kMlpP + 2 * 4 * (size_t)cmp::kMlpMaxRows + kMlpP + (size_t)cmp::kMlpPartFloats;
    if (!c->mlp_dev) {
        if (hipMalloc(&c->mlp_dev, floats * sizeof(float)) != hipSuccess) {
            c->mlp_dev = nullptr;
            (void)hipGetLastError();
            return fail(c, CMP_ENOMEM, "network buffers");
        }
    }
    d->params = c->mlp_dev;
    d->m = d->params + kMlpP;
    d->v = d->m + kMlpP;
    d->X = d->v + kMlpP;
    d->Y = d->X + 4 * cmp::kMlpMaxRows;
    d->grad = d->Y + 4 * cmp::kMlpMaxRows;
    d->part = d->grad + kMlpP;
    return CMP_OK;
}

void stats(const float* X, int n, float* mu, float* sd) {
    for (int j = 0; j < 4; ++j) {
        double s = 0;
        for (int i = 0; i < n; ++i) s += X[4 * i + j];
        const double m = s / n;
        double q = 0;
        for (int i = 0; i < n; ++i) q += ((double)X[4 * i + j] - m) * ((double)X[4 * i + j] - m);
        const double d = std::sqrt(q / n);
        mu[j] = (float)m;
        sd[j] = d > 0 ? (float)d : 1.f;
    }
}

}  // namespace

int mlp_predict(cmp_ctx* c, int n, const float* Xraw, float* Yraw) {
    MlpDev d;
    int st = mlp_dev(c, &d);
    if (st) return st;
    if (c->mlp_params.size() != (size_t)kMlpP) return fail(c, CMP_ENODATA, "network has no parameters");
    HIP_TRY(c, hipMemcpyAsync(d.params, c->mlp_params.data(), kMlpP * 4, hipMemcpyHostToDevice, c->side));
    for (int off = 0; off < n; off += cmp::kMlpMaxRows) {
        const int cnt = std::min(n - off, cmp::kMlpMaxRows);
        std::vector<float> Xs(4 * (size_t)cnt);
        for (int i = 0; i < cnt; ++i)
            for (int j = 0; j < 4; ++j)
                Xs[4 * i + j] = (Xraw[4 * (size_t)(off + i) + j] - c->mu_x[j]) / c->sd_x[j];
        HIP_TRY(c, hipMemcpyAsync(d.X, Xs.data(), Xs.size() * 4, hipMemcpyHostToDevice, c->side));
        HIP_TRY(c, cmp::launch_mlp_infer(cnt, d.X, d.params, d.Y, c->side));
        HIP_TRY(c, hipMemcpyAsync(Yraw + 4 * (size_t)off, d.Y, 4 * (size_t)cnt * 4,
                                  hipMemcpyDeviceToHost, c->side));
        HIP_TRY(c, hipStreamSynchronize(c->side));
        for (int i = 0; i < cnt; ++i)
            for (int j = 0; j < 4; ++j) {
                float& y = Yraw[4 * (size_t)(off + i) + j];
                y = y * c->sd_y[j] + c->mu_y[j];
            }
    }
    return CMP_OK;
}

CMP_API int cmp_mlp_param_count(void) { return kMlpP; }

CMP_API int cmp_mlp_set_params(cmp_ctx* c, const float* p, int n) {
    if (!c || !p) return CMP_EINVAL;
    if (n != kMlpP) return fail(c, CMP_EINVAL, "expected %d parameters", kMlpP);
    c->mlp_params.assign(p, p + n);
    c->mlp_ready = true;
    c->cache.clear();
    return CMP_OK;
}

CMP_API int cmp_mlp_get_params(cmp_ctx* c, float* p, int n) {
    if (!c || !p) return CMP_EINVAL;
    if (n != kMlpP) return fail(c, CMP_EINVAL, "expected %d parameters", kMlpP);
    if (c->mlp_params.size() != (size_t)kMlpP) return fail(c, CMP_ENODATA, "network has no parameters");
    std::copy(c->mlp_params.begin(), c->mlp_params.end(), p);
    return CMP_OK;
}

CMP_API int cmp_mlp_set_norm(cmp_ctx* c, const float* mx, const float* sx, const float* my,
                             const float* sy) {
    if (!c || !mx || !sx || !my || !sy) return CMP_EINVAL;
    for (int j = 0; j < 4; ++j)
        if (!(sx[j] > 0) || !(sy[j] > 0)) return fail(c, CMP_EINVAL, "deviations must be > 0");
    std::copy(mx, mx + 4, c->mu_x);
    std::copy(sx, sx + 4, c->sd_x);
    std::copy(my, my + 4, c->mu_y);
    std::copy(sy, sy + 4, c->sd_y);
    c->cache.clear();
    return CMP_OK;
}

CMP_API int cmp_mlp_get_norm(cmp_ctx* c, float* mx, float* sx, float* my, float* sy) {
    if (!c || !mx || !sx || !my || !sy) return CMP_EINVAL;
    std::copy(c->mu_x, c->mu_x + 4, mx);
    std::copy(c->sd_x, c->sd_x + 4, sx);
    std::copy(c->mu_y, c->mu_y + 4, my);
    std::copy(c->sd_y, c->sd_y + 4, sy);
    return CMP_OK;
}

CMP_API int cmp_mlp_train(cmp_ctx* c, int n, const float* X, const float* Y, int steps, float lr,
                          float* loss_trace) {
    if (!c || !X || !Y) return CMP_EINVAL;
    if (n < 1 || n > cmp::kMlpMaxRows) return fail(c, CMP_EINVAL, "n must be 1..%d", cmp::kMlpMaxRows);
    if (steps < 0 || !(lr > 0)) return fail(c, CMP_EINVAL, "bad steps or lr");
    if (c->mlp_params.size() != (size_t)kMlpP) return fail(c, CMP_ENODATA, "set initial parameters first");
    MlpDev d;
    int st = mlp_dev(c, &d);
    if (st) return st;
    stats(X, n, c->mu_x, c->sd_x);
    stats(Y, n, c->mu_y, c->sd_y);
    std::vector<float> Xs(4 * (size_t)n), Ys(4 * (size_t)n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 4; ++j) {
            Xs[4 * i + j] = (X[4 * i + j] - c->mu_x[j]) / c->sd_x[j];
            Ys[4 * i + j] = (Y[4 * i + j] - c->mu_y[j]) / c->sd_y[j];
        }
    float* loss_dev = nullptr;
    if (steps > 0) HIP_TRY(c, hipMalloc(&loss_dev, (size_t)steps * 4));
    auto cleanup = [&]() {
        if (loss_dev) (void)hipFree(loss_dev);
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpyAsync(d.params, c->mlp_params.data(), kMlpP * 4, hipMemcpyHostToDevice, c->side);
    if (e == hipSuccess) e = hipMemcpyAsync(d.X, Xs.data(), Xs.size() * 4, hipMemcpyHostToDevice, c->side);
    if (e == hipSuccess) e = hipMemcpyAsync(d.Y, Ys.data(), Ys.size() * 4, hipMemcpyHostToDevice, c->side);
    if (e == hipSuccess) e = cmp::launch_mlp_train(n, d.X, d.Y, d.params, d.m, d.v, d.part, steps, 0, lr, loss_dev, nullptr, c->side);
    if (e == hipSuccess) e = hipMemcpyAsync(c->mlp_params.data(), d.params, kMlpP * 4, hipMemcpyDeviceToHost, c->side);
    if (e == hipSuccess && loss_trace && steps > 0)
        e = hipMemcpyAsync(loss_trace, loss_dev, (size_t)steps * 4, hipMemcpyDeviceToHost, c->side);
    if (e == hipSuccess) e = hipStreamSynchronize(c->side);
    cleanup();
    if (e != hipSuccess) return hip_fail(c, e, "network training");
    c->mlp_ready = true;
    c->cache.clear();
    return CMP_OK;
}

CMP_API int cmp_mlp_grad(cmp_ctx* c, int n, const float* Xs, const float* Ys, float* loss,
                         float* grad) {
    if (!c || !Xs || !Ys || !grad) return CMP_EINVAL;
    if (n < 1 || n > cmp::kMlpMaxRows) return fail(c, CMP_EINVAL, "n must be 1..%d", cmp::kMlpMaxRows);
    if (c->mlp_params.size() != (size_t)kMlpP) return fail(c, CMP_ENODATA, "set parameters first");
    MlpDev d;
    int st = mlp_dev(c, &d);
    if (st) return st;
    float* scratch = nullptr;  // one float: the loss
    HIP_TRY(c, hipMalloc(&scratch, 4));
    hipError_t e = hipMemcpyAsync(d.params, c->mlp_params.data(), kMlpP * 4, hipMemcpyHostToDevice, c->side);
    if (e == hipSuccess) e = hipMemcpyAsync(d.X, Xs, 4 * (size_t)n * 4, hipMemcpyHostToDevice, c->side);
    if (e == hipSuccess) e = hipMemcpyAsync(d.Y, Ys, 4 * (size_t)n * 4, hipMemcpyHostToDevice, c->side);
    if (e == hipSuccess) e = cmp::launch_mlp_train(n, d.X, d.Y, d.params, d.m, d.v, d.part, 0, 0, 0.f, scratch, d.grad, c->side);
    if (e == hipSuccess) e = hipMemcpyAsync(grad, d.grad, kMlpP * 4, hipMemcpyDeviceToHost, c->side);
    float h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, scratch, 4, hipMemcpyDeviceToHost, c->side);
    if (e == hipSuccess) e = hipStreamSynchronize(c->side);
    (void)hipFree(scratch);
    if (e != hipSuccess) return hip_fail(c, e, "network gradient");
    if (loss) *loss = h;
    return CMP_OK;
}

CMP_API int cmp_mlp_infer(cmp_ctx* c, int n, const float* Xs, float* Yout) {
    if (!c || !Xs || !Yout) return CMP_EINVAL;
    if (n < 0) return fail(c, CMP_EINVAL, "n must be >= 0");
    if (c->mlp_params.size() != (size_t)kMlpP) return fail(c, CMP_ENODATA, "set parameters first");
    MlpDev d;
    int st = mlp_dev(c, &d);
    if (st) return st;
    HIP_TRY(c, hipMemcpyAsync(d.params, c->mlp_params.data(), kMlpP * 4, hipMemcpyHostToDevice, c->side));
    for (int off = 0; off < n; off += cmp::kMlpMaxRows) {
        const int cnt = std::min(n - off, cmp::kMlpMaxRows);
        HIP_TRY(c, hipMemcpyAsync(d.X, Xs + 4 * (size_t)off, 4 * (size_t)cnt * 4, hipMemcpyHostToDevice, c->side));
        HIP_TRY(c, cmp::launch_mlp_infer(cnt, d.X, d.params, d.Y, c->side));
        HIP_TRY(c, hipMemcpyAsync(Yout + 4 * (size_t)off, d.Y, 4 * (size_t)cnt * 4, hipMemcpyDeviceToHost, c->side));
    }
    HIP_TRY(c, hipStreamSynchronize(c->side));
    return CMP_OK;
}

CMP_API int cmp_mlp_fit_history(cmp_ctx* c, int steps, float lr, uint64_t seed, float* final_loss) {
    if (!c) return CMP_EINVAL;
    if (!c->gpu) return fail(c, CMP_EUNSUPPORTED, "learned selector needs a GPU context");
    Interface* f = find_iface(c, kGemm);
    if ((int)f->variants.size() < kNumBuiltin) return fail(c, CMP_ENODATA, "built-in variants missing");
    ShapeTable T = shape_table(c, f->variants.size());
    std::vector<float> X, Y;
    int n = 0;
    for (size_t s = 0; s < T.shapes.size() && n < cmp::kMlpMaxRows; ++s) {
        bool complete = true;
        for (int i = 0; i < kNumBuiltin; ++i)
            if (!std::isfinite(T.med[s][i])) complete = false;
        if (!complete) continue;
        const double tol = kTolClasses[splitmix64_at(seed, (uint64_t)n) % 3];
        X.push_back((float)std::log2((double)std::get<0>(T.shapes[s])));
        X.push_back((float)std::log2((double)std::get<1>(T.shapes[s])));
        X.push_back((float)std::log2((double)std::get<2>(T.shapes[s])));
        X.push_back((float)std::log10(tol));
        for (int i = 0; i < kNumBuiltin; ++i) Y.push_back((float)std::log(T.med[s][i] * 1000.0));
        ++n;
    }
    if (n < 2) return fail(c, CMP_ENODATA, "history holds fewer than 2 fully timed shapes");
    // Kaiming-uniform initialisation from splitmix64(seed ^ golden)
    std::vector<float> p;
    const int sizes[4] = {4, 64, 64, 4};
    uint64_t j = 0;
    const uint64_t s2 = seed ^ 0x9e3779b97f4a7c15ull;
    for (int l = 0; l < 3; ++l) {
        const int fi = sizes[l], fo = sizes[l + 1];
        const double wb = std::sqrt(6.0 / fi), bb = 1.0 / std::sqrt((double)fi);
        for (int i = 0; i < fo * fi; ++i) p.push_back((float)((2 * u01(splitmix64_at(s2, j++)) - 1) * wb));
        for (int i = 0; i < fo; ++i) p.push_back((float)((2 * u01(splitmix64_at(s2, j++)) - 1) * bb));
    }
    c->mlp_params = p;
    std::vector<float> trace(std::max(steps, 1));
    int st = cmp_mlp_train(c, n, X.data(), Y.data(), steps, lr, trace.data());
    if (st) return st;
    if (final_loss) *final_loss = steps > 0 ? trace[steps - 1] : 0.f;
    return CMP_OK;
}

CMP_API int cmp_mlp_save(cmp_ctx* c, const char* path) {
    if (!c || !path) return CMP_EINVAL;
    if (c->mlp_params.size() != (size_t)kMlpP) return fail(c, CMP_ENODATA, "network has no parameters");
    std::ofstream o(path);
    if (!o) return fail(c, CMP_EINVAL, "cannot open %s", path);
    o << "# compar-mlp v1\n";
    o << "# device " << device_signature(c) << "\n";
    o << "# lib " << kVersion << "\n";
    char buf[32];
    auto row = [&](const char* name, const float* v, int n) {
        o << name;
        for (int i = 0; i < n; ++i) {
            std::snprintf(buf, sizeof buf, " %.9g", v[i]);
            o << buf;
        }
        o << "\n";
    };
    row("mu_x", c->mu_x, 4);
    row("sd_x", c->sd_x, 4);
    row("mu_y", c->mu_y, 4);
    row("sd_y", c->sd_y, 4);
    row("params", c->mlp_params.data(), kMlpP);
    if (!o) return fail(c, CMP_EINVAL, "write to %s failed", path);
    return CMP_OK;
}

CMP_API int cmp_mlp_load(cmp_ctx* c, const char* path, int force) {
    if (!c || !path) return CMP_EINVAL;
    std::ifstream in(path);
    if (!in) return fail(c, CMP_EINVAL, "cannot open %s", path);
    std::string line;
    bool header = false;
    std::map<std::string, std::vector<float>> rows;
    while (std::getline(in, line)) {
        if (line.empty()) continue;
        if (line[0] == '#') {
            if (line.rfind("# compar-mlp v1", 0) == 0) header = true;
            if (line.rfind("# device ", 0) == 0 && !force) {
                const std::string sig = line.substr(9);
                if (sig != device_signature(c))
                    return fail(c, CMP_EINVAL, "network saved on '%s', this device is '%s'", sig.c_str(),
                                device_signature(c).c_str());
            }
            continue;
        }
        std::istringstream ss(line);
        std::string name;
        ss >> name;
        std::vector<float> v;
        std::string tok;
        while (ss >> tok) {
            char* end = nullptr;
            const float x = std::strtof(tok.c_str(), &end);
            if (!end || *end) return fail(c, CMP_EINVAL, "malformed value '%s' in %s", tok.c_str(), path);
            v.push_back(x);
        }
        rows[name] = std::move(v);
    }
    if (!header) return fail(c, CMP_EINVAL, "%s is not a compar network file", path);
    for (const char* k : {"mu_x", "sd_x", "mu_y", "sd_y"})
        if (rows[k].size() != 4) return fail(c, CMP_EINVAL, "%s: %s needs 4 values", path, k);
    if (rows["params"].size() != (size_t)kMlpP)
        return fail(c, CMP_EINVAL, "%s holds %zu parameters, the network has %d", path, rows["params"].size(), kMlpP);
    for (const char* k : {"mu_x", "sd_x", "mu_y", "sd_y", "params"})
        for (float x : rows[k])
            if (!std::isfinite(x)) return fail(c, CMP_EINVAL, "%s: %s holds a non-finite value", path, k);
    for (int j = 0; j < 4; ++j)
        if (!(rows["sd_x"][j] > 0) || !(rows["sd_y"][j] > 0))
            return fail(c, CMP_EINVAL, "%s: deviations must be > 0", path);
    std::copy(rows["mu_x"].begin(), rows["mu_x"].end(), c->mu_x);
    std::copy(rows["sd_x"].begin(), rows["sd_x"].end(), c->sd_x);
    std::copy(rows["mu_y"].begin(), rows["mu_y"].end(), c->mu_y);
    std::copy(rows["sd_y"].begin(), rows["sd_y"].end(), c->sd_y);
    c->mlp_params = rows["params"];
    c->mlp_ready = true;
    c->cache.clear();
    return CMP_OK;
}

// ---------------------------------------------------------------------------
// Verification and pre-pass entry points

CMP_API int cmp_freivalds(cmp_ctx* c, const cmp_gemm_args* a, const float* c0, const double* x,
                          void* stream, double* est) {
    if (!c || !est || !x) return CMP_EINVAL;
    if (!c->gpu) return fail(c, CMP_EUNSUPPORTED, "needs a GPU context");
    int st = check_gemm_args(c, a);
    if (st) return st;
    if (a->M == 0 || a->N == 0) {
        *est = 0;
        return CMP_OK;
    }
    if (a->beta != 0.f && !c0) return fail(c, CMP_EINVAL, "beta != 0 needs the old C");
    auto s = (hipStream_t)stream;
    const VLayout L = vlayout(a, false);
    st = ensure_vws(c, L.total_b);
    if (st) return st;
    double* xdev = (double*)c->vws + L.x_d;
    HIP_TRY(c, hipMemcpyAsync(xdev, x, (size_t)a->N * 8, hipMemcpyHostToDevice, s));
    return probe(c, a, c0, a->ldc, xdev, s, est);
}

CMP_API int cmp_last_verify(cmp_ctx* c, double* est, int* fallbacks) {
    if (!c) return CMP_EINVAL;
    if (est) *est = c->last_verify;
    if (fallbacks) *fallbacks = c->fallbacks;
    return CMP_OK;
}

CMP_API int cmp_split_bf16(cmp_ctx* c, int64_t rows, int64_t cols, const float* X, int64_t ldx,
                           uint16_t* hi, uint16_t* lo, void* stream) {
    if (!c) return CMP_EINVAL;
    if (!c->gpu) return fail(c, CMP_EUNSUPPORTED, "needs a GPU context");
    if (rows < 0 || cols < 0 || ldx < std::max<int64_t>(cols, 1)) return fail(c, CMP_EINVAL, "bad shape");
    if (rows == 0 || cols == 0) return CMP_OK;
    if (!X || !hi) return fail(c, CMP_EINVAL, "null pointer");
    HIP_TRY(c, cmp::launch_split_bf16_plain(rows, cols, X, ldx, hi, lo, (hipStream_t)stream));
    return CMP_OK;
}

CMP_API int cmp_quant_fp8(cmp_ctx* c, int64_t rows, int64_t cols, const float* X, int64_t ldx,
                          uint8_t* q, uint8_t* qs, uint8_t* rq, uint8_t* rs, void* stream) {
    if (!c) return CMP_EINVAL;
    if (!c->gpu) return fail(c, CMP_EUNSUPPORTED, "needs a GPU context");
    if (rows < 0 || cols < 0 || ldx < std::max<int64_t>(cols, 1)) return fail(c, CMP_EINVAL, "bad shape");
    if (rows == 0 || cols == 0) return CMP_OK;
    if (!X || !q || !qs || !rq || !rs) return fail(c, CMP_EINVAL, "null pointer");
    if ((rows % 128) || (cols % 128)) {
        // outputs are tight: the kernel writes whole 128 x 128 tiles, so ragged
        // extents go through a padded staging image in the workspace
        const int64_t rp = round_up(rows, 128), cp = round_up(cols, 128);
        const size_t need = 2 * (size_t)rp * cp + 2 * (size_t)(rp / 128) * (cp / 128);
        int st = ensure_ws(c, need);
        if (st) return st;
        auto* q2 = (uint8_t*)c->ws;
        auto* r2 = q2 + (size_t)rp * cp;
        auto* s1 = r2 + (size_t)rp * cp;
        auto* s2 = s1 + (size_t)(rp / 128) * (cp / 128);
        auto s = (hipStream_t)stream;
        HIP_TRY(c, cmp::launch_quant_fp8(rows, cols, X, ldx, false, false, rp, cp, q2, s1, r2, s2, s));
        HIP_TRY(c, hipMemcpy2DAsync(q, cols, q2, cp, cols, rows, hipMemcpyDeviceToDevice, s));
        HIP_TRY(c, hipMemcpy2DAsync(rq, cols, r2, cp, cols, rows, hipMemcpyDeviceToDevice, s));
        HIP_TRY(c, hipMemcpyAsync(qs, s1, (size_t)(rp / 128) * (cp / 128), hipMemcpyDeviceToDevice, s));
        HIP_TRY(c, hipMemcpyAsync(rs, s2, (size_t)(rp / 128) * (cp / 128), hipMemcpyDeviceToDevice, s));
        return CMP_OK;
    }
    HIP_TRY(c, cmp::launch_quant_fp8(rows, cols, X, ldx, false, false, rows, cols, q, qs, rq, rs,
                                     (hipStream_t)stream));
    return CMP_OK;
}

CMP_API int cmp_quant_mx6(cmp_ctx* c, int64_t rows, int64_t cols, const float* X, int64_t ldx,
                          int transpose, uint8_t* q, uint8_t* qs, uint8_t* rq, uint8_t* rs,
                          void* stream) {
    if (!c) return CMP_EINVAL;
    if (!c->gpu) return fail(c, CMP_EUNSUPPORTED, "needs a GPU context");
    if (rows < 0 || cols < 0 || ldx < std::max<int64_t>(cols, 1)) return fail(c, CMP_EINVAL, "bad shape");
    if (rows == 0 || cols == 0) return CMP_OK;
    if (!X || !q || !qs || !rq || !rs) return fail(c, CMP_EINVAL, "null pointer");
    HIP_TRY(c, cmp::launch_quant_mx6(rows, cols, X, ldx, transpose != 0, false, 0, 0, q, qs, rq, rs,
                                     (hipStream_t)stream));
    return CMP_OK;
}

CMP_API int cmp_prepass_layout(cmp_ctx* c, int id, int64_t M, int64_t N, int64_t K,
                               cmp_image_layout* out) {
    if (!c || !out || M < 1 || N < 1 || K < 1) return CMP_EINVAL;
    Interface* f = find_iface(c, kGemm);
    if (!f || id < 0 || id >= (int)f->variants.size()) return fail(c, CMP_EINVAL, "bad variant id %d", id);
    const int kind = image_kind(f->variants[id]);
    if (kind == kImgNone)
        return fail(c, CMP_EUNSUPPORTED, "variant %s has no operand pre-pass",
                    f->variants[id].name.c_str());
    const Images I = images_of(kind, M, N, K);
    *out = cmp_image_layout{};
    out->Mp = I.Mp;
    out->Np = I.Np;
    out->Kp = I.Kp;
    out->count = I.n;
    for (int i = 0; i < 8; ++i) {
        out->offset[i] = i < I.n ? (int64_t)I.off[i] : -1;
        out->bytes[i] = i < I.n ? (int64_t)I.bytes[i] : 0;
    }
    out->total = (int64_t)I.total;
    return CMP_OK;
}

CMP_API int cmp_prepass_images(cmp_ctx* c, int id, const cmp_gemm_args* a, void* out,
                               size_t out_bytes, void* stream) {
    if (!c || !a) return CMP_EINVAL;
    if (!c->gpu) return fail(c, CMP_EUNSUPPORTED, "needs a GPU context");
    cmp_image_layout L;
    int st = cmp_prepass_layout(c, id, a->M, a->N, a->K, &L);
    if (st) return st;
    if (!a->A || !a->B || !out) return fail(c, CMP_EINVAL, "null pointer");
    if (a->lda < a->K || a->ldb < a->N) return fail(c, CMP_EINVAL, "lda < K or ldb < N");
    if (out_bytes < (size_t)L.total)
        return fail(c, CMP_EINVAL, "image buffer of %zu bytes, %lld needed", out_bytes,
                    (long long)L.total);
    Interface* f = find_iface(c, kGemm);
    const int kind = image_kind(f->variants[id]);
    st = prepass(c, kind, a, images_of(kind, a->M, a->N, a->K), out, (hipStream_t)stream);
    if (st == CMP_EHIP) return hip_fail(c, hipGetLastError(), "pre-pass launch");
    return st;
}

// ---------------------------------------------------------------------------
// Per-kernel timing of the built-in variants

CMP_API int cmp_kernel_timing(cmp_ctx* c, int enable) {
    if (!c) return CMP_EINVAL;
    if (!c->gpu) return fail(c, CMP_EUNSUPPORTED, "needs a GPU context");
    c->ktime = enable != 0;
    return CMP_OK;
}

CMP_API int cmp_kernel_stats(cmp_ctx* c, int idx, char* name, size_t name_len, long long* launches,
                             double* total_ms) {
    if (!c) return CMP_EINVAL;
    // fold completed event pairs into the totals (waits for the recorded events)
    for (auto& k : c->kpending) {
        float ms = 0;
        if (hipEventSynchronize(k.b) == hipSuccess && hipEventElapsedTime(&ms, k.a, k.b) == hipSuccess) {
            auto& st = c->kstats[k.name];
            st.first += 1;
            st.second += ms;
        }
        c->kpool.push_back(k.a);
        c->kpool.push_back(k.b);
    }
    c->kpending.clear();
    if (idx < 0) {  // reset
        c->kstats.clear();
        return CMP_OK;
    }
    if (idx >= (int)c->kstats.size()) return CMP_ENOTFOUND;
    auto it = c->kstats.begin();
    std::advance(it, idx);
    if (name && name_len) std::snprintf(name, name_len, "%s", it->first.c_str());
    if (launches) *launches = it->second.first;
    if (total_ms) *total_ms = it->second.second;
    return CMP_OK;
}

// ---------------------------------------------------------------------------
// Grouped launches: many GEMMs of uneven shapes in one persistent kernel

struct cmp_grouped_plan {
    cmp_ctx* ctx = nullptr;
    int count = 0;           // problems with at least one tile
    int config = -1;
    int total_tiles = 0;
    int grid = 0;
    cmp::GroupedDesc* desc = nullptr;     // device: the descriptors, then the tile-queue counter
    cmp::GroupedMfmaDesc* mdesc = nullptr;   // the same for the bf16x3 configuration
    void* images = nullptr;               // device: that configuration's bf16 hi / lo images
    int64_t pre_total = 0;                // its pre-pass workgroups
    unsigned* counter = nullptr;          // device, inside the descriptor allocation
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<float> config_ms;         // autotuner medians per configuration (NaN: not tried)
};

namespace {

// Descriptors for one tile configuration.  A tile's time grows with its
// problem's K, so problems go in decreasing order of K (then of M x N): the
// kernel hands tiles out greedily in list order, and serving the longest
// tiles first keeps the finishing times of the workgroups close together.
int build_descs(cmp_ctx* c, const std::vector<cmp_gemm_args>& probs, int config,
                std::vector<cmp::GroupedDesc>* out, int* total) {
    const int bm = cmp::kGroupedConfigs[config].bm, bn = cmp::kGroupedConfigs[config].bn;
    std::vector<int> order;
    for (int i = 0; i < (int)probs.size(); ++i)
        if (probs[i].M > 0 && probs[i].N > 0) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        if (probs[x].K != probs[y].K) return probs[x].K > probs[y].K;
        return (double)probs[x].M * probs[x].N > (double)probs[y].M * probs[y].N;
    });
    out->clear();
    int64_t start = 0;
    for (int i : order) {
        const cmp_gemm_args& a = probs[i];
        cmp::GroupedDesc d{};
        d.M = a.M; d.N = a.N; d.K = a.K;
        d.lda = a.lda; d.ldb = a.ldb; d.ldc = a.ldc;
        d.alpha = a.alpha; d.beta = a.beta;
        d.A = a.A; d.B = a.B; d.C = a.C;
        const int64_t tm = (a.M + bm - 1) / bm, tn = (a.N + bn - 1) / bn;
        d.tiles_n = (int)tn;
        d.tile_start = (int)start;
        d.vec = (a.lda % 4 == 0) && (a.ldb % 4 == 0) && ((reinterpret_cast<uintptr_t>(a.A) & 15) == 0) &&
                ((reinterpret_cast<uintptr_t>(a.B) & 15) == 0);
        start += tm * tn;
        if (start > INT32_MAX) return fail(c, CMP_EINVAL, "grouped launch exceeds 2^31 tiles");
        out->push_back(d);
    }
    *total = (int)start;
    return CMP_OK;
}

int upload_descs(cmp_ctx* c, cmp_grouped_plan* pl, const std::vector<cmp::GroupedDesc>& d,
                 hipStream_t s) {
    if (pl->desc) HIP_TRY(c, hipFree(pl->desc));
    pl->desc = nullptr;
    pl->counter = nullptr;
    const size_t dbytes = (size_t)round_up((int64_t)(std::max<size_t>(d.size(), 1) * sizeof(cmp::GroupedDesc)), 256);
    HIP_TRY(c, hipMalloc(&pl->desc, dbytes + 256));
    pl->counter = reinterpret_cast<unsigned*>(reinterpret_cast<uint8_t*>(pl->desc) + dbytes);
    if (!d.empty())
        HIP_TRY(c, hipMemcpyAsync(pl->desc, d.data(), d.size() * sizeof(cmp::GroupedDesc),
                                  hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    return CMP_OK;
}

int grouped_grid(cmp_ctx* c, int config, int total_tiles) {
    const int per_cu = cmp::grouped_blocks_per_cu(config);
    return std::max(1, std::min(total_tiles, per_cu * c->props.multiProcessorCount));
}

// The configurations after the FP32 SIMT tiles: kGroupedMfma runs every
// problem with the bf16x3 variant's arithmetic (its pre-pass and its 256 x 256
// MFMA tile), bit-identical to one unsplit bf16x3 call per problem.
constexpr int kGroupedMfma = cmp::kNumGroupedConfigs;
constexpr int kGroupedAll = kGroupedMfma + 1;

// The bf16x3 configuration needs every problem to read A and B: alpha == 0 or
// K == 0 (C = beta C, operands never read) is left to the SIMT configurations.
bool mfma_eligible(const std::vector<cmp_gemm_args>& probs) {
    for (const auto& a : probs)
        if (a.M > 0 && a.N > 0 && (a.alpha == 0.f || a.K == 0)) return false;
    return true;
}

void free_plan_buffers(cmp_grouped_plan* pl) {
    if (pl->desc) (void)hipFree(pl->desc);
    if (pl->mdesc) (void)hipFree(pl->mdesc);
    if (pl->images) (void)hipFree(pl->images);
    pl->desc = nullptr;
    pl->mdesc = nullptr;
    pl->images = nullptr;
    pl->counter = nullptr;
    pl->pre_total = 0;
}

// Descriptors, images and counter of the bf16x3 configuration (problem order
// as in build_descs).
int build_mfma(cmp_ctx* c, cmp_grouped_plan* pl, const std::vector<cmp_gemm_args>& probs, hipStream_t s) {
    std::vector<int> order;
    for (int i = 0; i < (int)probs.size(); ++i)
        if (probs[i].M > 0 && probs[i].N > 0) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        if (probs[x].K != probs[y].K) return probs[x].K > probs[y].K;
        return (double)probs[x].M * probs[x].N > (double)probs[y].M * probs[y].N;
    });
    std::vector<cmp::GroupedMfmaDesc> d;
    std::vector<size_t> img_off;              // per problem: offset of its four images
    size_t img_bytes = 0;
    int64_t pre = 0, tiles = 0;
    for (int i : order) {
        const cmp_gemm_args& a = probs[i];
        cmp::GroupedMfmaDesc g{};
        g.M = a.M; g.N = a.N; g.K = a.K;
        g.lda = a.lda; g.ldb = a.ldb; g.ldc = a.ldc;
        g.Mp = round_up(a.M, cmp::kMfmaTileM);
        g.Np = round_up(a.N, cmp::kMfmaTileN);
        g.Kp = round_up(a.K, cmp::kBf16TileK);
        g.alpha = a.alpha; g.beta = a.beta;
        g.A = a.A; g.B = a.B; g.C = a.C;
        // A: one workgroup per 64-row quarter of a 256-row x 64-byte block below M
        g.ga = (int)((a.M / 256 * 4 + (a.M % 256 + 63) / 64) * (g.Kp * 2 / 64));
        g.gb = (int)(((a.N + 63) / 64) * (g.Kp / 64));   // the 64-row tiles of B^T below N
        g.pre_start = (int)pre;
        g.tile_start = (int)tiles;
        g.tiles_n = (int)(g.Np / cmp::kMfmaTileN);
        g.vec = ((a.lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(a.A) & 15) == 0) ? 1 : 0) |
                ((a.ldb % 4 == 0) && ((reinterpret_cast<uintptr_t>(a.B) & 15) == 0) ? 2 : 0);
        pre += (int64_t)g.ga + g.gb;
        tiles += (g.Mp / cmp::kMfmaTileM) * (g.Np / cmp::kMfmaTileN);
        // (a workgroup's copy offsets reach its panel's K blocks: 64 bytes of K x 256 rows each)
        if (pre > INT32_MAX || tiles > INT32_MAX || g.Kp * 2 / 64 * 16384 > INT32_MAX)
            return fail(c, CMP_EINVAL, "grouped bf16x3 launch too large");
        img_off.push_back(img_bytes);
        img_bytes += (size_t)round_up(g.Mp * g.Kp * 2, 256) * 2 + (size_t)round_up(g.Np * g.Kp * 2, 256) * 2;
        d.push_back(g);
    }
    if (img_bytes) HIP_TRY(c, hipMalloc(&pl->images, img_bytes));
    for (size_t p = 0; p < d.size(); ++p) {
        uint8_t* base = reinterpret_cast<uint8_t*>(pl->images) + img_off[p];
        const size_t as = (size_t)round_up(d[p].Mp * d[p].Kp * 2, 256), bs = (size_t)round_up(d[p].Np * d[p].Kp * 2, 256);
        d[p].ah = reinterpret_cast<uint16_t*>(base);
        d[p].al = reinterpret_cast<uint16_t*>(base + as);
        d[p].bh = reinterpret_cast<uint16_t*>(base + 2 * as);
        d[p].bl = reinterpret_cast<uint16_t*>(base + 2 * as + bs);
    }
    const size_t dbytes = (size_t)round_up((int64_t)(std::max<size_t>(d.size(), 1) * sizeof(cmp::GroupedMfmaDesc)), 256);
    HIP_TRY(c, hipMalloc(&pl->mdesc, dbytes + 256));
    pl->counter = reinterpret_cast<unsigned*>(reinterpret_cast<uint8_t*>(pl->mdesc) + dbytes);
    if (!d.empty())
        HIP_TRY(c, hipMemcpyAsync(pl->mdesc, d.data(), d.size() * sizeof(cmp::GroupedMfmaDesc),
                                  hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    pl->count = (int)d.size();
    pl->total_tiles = (int)tiles;
    pl->pre_total = pre;
    pl->grid = std::max(1, std::min((int)tiles, c->props.multiProcessorCount));   // one 128 KiB ring per CU
    return CMP_OK;
}

// Buffers and launch shape of configuration cfg (the previous ones freed).
int setup_config(cmp_ctx* c, cmp_grouped_plan* pl, const std::vector<cmp_gemm_args>& probs, int cfg,
                 hipStream_t s) {
    free_plan_buffers(pl);
    pl->config = cfg;
    if (cfg == kGroupedMfma) return build_mfma(c, pl, probs, s);
    std::vector<cmp::GroupedDesc> d;
    int total = 0, st;
    if ((st = build_descs(c, probs, cfg, &d, &total))) return st;
    if ((st = upload_descs(c, pl, d, s))) return st;
    pl->count = (int)d.size();
    pl->total_tiles = total;
    pl->grid = grouped_grid(c, cfg, total);
    return CMP_OK;
}

hipError_t plan_launch(cmp_grouped_plan* pl, hipStream_t s) {
    if (pl->config == kGroupedMfma) {
        hipError_t e = cmp::launch_split_grouped(pl->mdesc, pl->count, pl->pre_total, s);
        if (e == hipSuccess)
            e = cmp::launch_gemm_bf16x3_grouped(pl->mdesc, pl->count, pl->total_tiles, pl->grid, pl->counter, s);
        return e;
    }
    return cmp::launch_gemm_f32_grouped(pl->config, pl->desc, pl->count, pl->total_tiles, pl->grid,
                                        pl->counter, s);
}

}  // namespace

CMP_API int cmp_grouped_config_count(void) { return kGroupedAll; }

CMP_API int cmp_grouped_config_info(int config, int* bm, int* bn, int* bk) {
    if (config < 0 || config >= kGroupedAll) return CMP_EINVAL;
    if (config == kGroupedMfma) {
        if (bm) *bm = cmp::kMfmaTileM;
        if (bn) *bn = cmp::kMfmaTileN;
        if (bk) *bk = 32;                  // bf16 values per 64-byte K block of the images
        return CMP_OK;
    }
    if (bm) *bm = cmp::kGroupedConfigs[config].bm;
    if (bn) *bn = cmp::kGroupedConfigs[config].bn;
    if (bk) *bk = cmp::kGroupedConfigs[config].bk;
    return CMP_OK;
}

CMP_API int cmp_grouped_config_variant(int config, int* variant) {
    if (config < 0 || config >= kGroupedAll || !variant) return CMP_EINVAL;
    *variant = config == kGroupedMfma ? 1 : 0;     // built-in ids: 0 f32_simt, 1 bf16x3
    return CMP_OK;
}

CMP_API int cmp_grouped_plan_create(cmp_ctx* c, int count, const cmp_gemm_args* probs, int config,
                                    int reps, void* stream, cmp_grouped_plan** out) {
    if (!c || !out) return CMP_EINVAL;
    *out = nullptr;
    if (!c->gpu) return fail(c, CMP_EUNSUPPORTED, "needs a GPU context");
    if (count < 0 || (count > 0 && !probs)) return fail(c, CMP_EINVAL, "bad problem list");
    if (config >= kGroupedAll) return fail(c, CMP_EINVAL, "unknown tile configuration %d", config);
    if (reps < 1) return fail(c, CMP_EINVAL, "reps must be >= 1");
    std::vector<cmp_gemm_args> pv(probs, probs + count);
    for (int i = 0; i < count; ++i) {
        int st = check_gemm_args(c, &pv[i]);
        if (st) return fail(c, st, "problem %d: %s", i, c->last_error.c_str());
    }
    const bool mfma_ok = mfma_eligible(pv);
    if (config == kGroupedMfma && !mfma_ok)
        return fail(c, CMP_EUNSUPPORTED, "the bf16x3 configuration needs alpha != 0 and K > 0 in every problem");
    auto s = (hipStream_t)stream;
    auto* pl = new (std::nothrow) cmp_grouped_plan();
    if (!pl) return fail(c, CMP_ENOMEM, "plan");
    pl->ctx = c;
    pl->config_ms.assign(kGroupedAll, NAN);
    auto cleanup = [&](int st) {
        free_plan_buffers(pl);
        delete pl;
        return st;
    };
    int st;
    if (config < 0) {
        // autotuner: time every configuration on this very group (the bf16x3 one with
        // its pre-pass) and keep the fastest
        hipEvent_t e0, e1;
        HIP_TRY(c, hipEventCreate(&e0));
        HIP_TRY(c, hipEventCreate(&e1));
        float best = INFINITY;
        int best_cfg = 0;
        for (int cfg = 0; cfg < kGroupedAll; ++cfg) {
            if (cfg == kGroupedMfma && !mfma_ok) continue;
            if ((st = setup_config(c, pl, pv, cfg, s))) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return cleanup(st);
            }
            std::vector<float> t(reps);
            hipError_t he = plan_launch(pl, s);
            for (int r = 0; r < reps && he == hipSuccess; ++r) {
                (void)hipEventRecord(e0, s);
                he = plan_launch(pl, s);
                (void)hipEventRecord(e1, s);
                if (he == hipSuccess) he = hipEventSynchronize(e1);
                if (he == hipSuccess) he = hipEventElapsedTime(&t[r], e0, e1);
            }
            if (he != hipSuccess) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return cleanup(hip_fail(c, he, "grouped autotune"));
            }
            std::sort(t.begin(), t.end());
            pl->config_ms[cfg] = t[reps / 2];
            if (t[reps / 2] < best) {
                best = t[reps / 2];
                best_cfg = cfg;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        config = best_cfg;
    }
    if ((st = setup_config(c, pl, pv, config, s))) return cleanup(st);
    // capture the launch into a graph on a private stream
    hipStream_t cap = nullptr;
    hipError_t he = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (he == hipSuccess) {
        hipError_t le = plan_launch(pl, cap);
        he = hipStreamEndCapture(cap, &pl->graph);
        if (he == hipSuccess) he = le;
    }
    if (he == hipSuccess) he = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
    if (cap) (void)hipStreamDestroy(cap);
    if (he != hipSuccess) {
        if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
        if (pl->graph) (void)hipGraphDestroy(pl->graph);
        return cleanup(hip_fail(c, he, "grouped graph capture"));
    }
    *out = pl;
    return CMP_OK;
}

CMP_API int cmp_grouped_plan_info(const cmp_grouped_plan* pl, int* config, int* problems, int* tiles,
                                  int* grid, float* config_ms) {
    if (!pl) return CMP_EINVAL;
    if (config) *config = pl->config;
    if (problems) *problems = pl->count;
    if (tiles) *tiles = pl->total_tiles;
    if (grid) *grid = pl->grid;
    if (config_ms)
        for (int i = 0; i < kGroupedAll; ++i) config_ms[i] = pl->config_ms[i];
    return CMP_OK;
}

CMP_API int cmp_grouped_launch(cmp_grouped_plan* pl, void* stream) {
    if (!pl) return CMP_EINVAL;
    cmp_ctx* c = pl->ctx;
    HIP_TRY(c, plan_launch(pl, (hipStream_t)stream));
    return CMP_OK;
}

CMP_API int cmp_grouped_graph_launch(cmp_grouped_plan* pl, void* stream) {
    if (!pl) return CMP_EINVAL;
    cmp_ctx* c = pl->ctx;
    HIP_TRY(c, hipGraphLaunch(pl->exec, (hipStream_t)stream));
    return CMP_OK;
}

CMP_API int cmp_grouped_plan_destroy(cmp_grouped_plan* pl) {
    if (!pl) return CMP_OK;
    (void)hipDeviceSynchronize();
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    free_plan_buffers(pl);
    delete pl;
    return CMP_OK;
}

// CPU stand-ins for the HIP runtime calls and the kernel launch layer (dk::launch_* and the
// capability queries) that the host driver uses, for a sanitizer build of the dk_*.cpp sources without a
// GPU.  Test infrastructure only.
//
// Each stand-in kernel touches exactly the buffer extents the real kernel reads and writes
// (first and last byte and one byte per 4 KiB page in between, so that AddressSanitizer sees any
// out-of-range extent or freed buffer), and produces per-sample values that are a pure function
// of (seed, tag, level, sample, observable): fake_value() below, which the harness recomputes on
// its own to check the driver's chunking, ordering and merging.  The streaming stand-ins carry
// the identity of the sample and its step count in the first words of each sample's state and
// check, at every launch, that the state they are handed belongs to the sample they are told to
// advance and continues at the step they are told to start from.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "../../../paper_2311_08872_amd/csrc/dk_cnn.h"
#include "../../../paper_2311_08872_amd/csrc/dk_fourier.h"
#include "../../../paper_2311_08872_amd/csrc/dk_internal.h"
#include "../../../paper_2311_08872_amd/csrc/dk_round.h"
#include "../../../paper_2311_08872_amd/csrc/dk_stream.h"
#include "../../../paper_2311_08872_amd/csrc/dk_theta.h"

// ------------------------------------------------------------------------------------------
// Errors found by the stand-ins; the harness fails when any were recorded.
// ------------------------------------------------------------------------------------------
std::vector<std::string> g_fake_errors;
uint64_t g_fake_launches = 0;
uint64_t g_fake_graph_launches = 0;

static void fake_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
static void fake_error(const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (g_fake_errors.size() < 64) g_fake_errors.push_back(buf);
}

// ------------------------------------------------------------------------------------------
// The per-sample values: level differences with mean 0.1 4^-l and variance 4^-l / 3 on
// pairs, P = 1 + (u - 1/2) on level 0 and on single paths; observable j scales them by 1 + j.
// ------------------------------------------------------------------------------------------
static uint64_t mix(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double unit(uint64_t seed, uint32_t tag, int level, uint64_t sample, int j, int k)
{
    uint64_t h = mix(seed ^ 0x1234567ull);
    h = mix(h ^ ((uint64_t)tag << 40) ^ ((uint64_t)level << 32) ^ (uint64_t)(j * 8 + k));
    h = mix(h ^ sample);
    return (double)(h >> 11) * 0x1.0p-53;
}

extern "C" double fake_value(uint64_t seed, uint32_t tag, int level, uint64_t sample, int j, int pair, int which)
{
    const double s = 1.0 + j;
    const double w = std::ldexp(1.0, -level);
    const double pf = 1.0 + w * (unit(seed, tag, level, sample, j, 0) - 0.5);
    if (!pair) return which == 0 ? s * pf : 0.0;
    const double y = 2.0 * w * (unit(seed, tag, level, sample, j, 1) - 0.5) + 0.1 * w * w;
    return which == 0 ? s * pf : s * (pf - y);
}

// ------------------------------------------------------------------------------------------
// Memory: "device" allocations are heap blocks filled with a pattern (device memory is not
// cleared), tracked so that a pointer that is not the start of a live device block is reported.
// ------------------------------------------------------------------------------------------
static std::map<const char*, size_t> g_dev;   // start -> bytes

static bool dev_range(const void* p, size_t bytes)
{
    if (bytes == 0) return true;
    const char* c = (const char*)p;
    auto it = g_dev.upper_bound(c);
    if (it == g_dev.begin()) return false;
    --it;
    return c >= it->first && c + bytes <= it->first + it->second;
}

static void touch_read(const void* p, size_t bytes, const char* what)
{
    if (bytes == 0) return;
    if (!p) { fake_error("%s: NULL pointer for %zu bytes", what, bytes); return; }
    if (!dev_range(p, bytes)) fake_error("%s: %zu bytes at %p are not inside one device allocation", what, bytes, p);
    const volatile char* c = (const volatile char*)p;
    char acc = 0;
    for (size_t i = 0; i < bytes; i += 4096) acc ^= c[i];
    acc ^= c[bytes - 1];
    (void)acc;
}

static void touch_write(void* p, size_t bytes, const char* what)
{
    if (bytes == 0) return;
    if (!p) { fake_error("%s: NULL pointer for %zu bytes", what, bytes); return; }
    if (!dev_range(p, bytes)) fake_error("%s: %zu bytes at %p are not inside one device allocation", what, bytes, p);
    volatile char* c = (volatile char*)p;
    for (size_t i = 0; i < bytes; i += 4096) c[i] = c[i];
    c[bytes - 1] = c[bytes - 1];
}

hipError_t hipMalloc(void** p, size_t bytes)
{
    if (!p) return hipErrorInvalidValue;
    char* b = (char*)std::malloc(bytes ? bytes : 1);
    if (!b) return hipErrorOutOfMemory;
    std::memset(b, 0xA5, bytes ? bytes : 1);
    g_dev[b] = bytes;
    *p = b;
    return hipSuccess;
}

hipError_t hipFree(void* p)
{
    if (!p) return hipSuccess;
    auto it = g_dev.find((const char*)p);
    if (it == g_dev.end()) { fake_error("hipFree of %p, not a device allocation", p); return hipErrorInvalidValue; }
    g_dev.erase(it);
    std::free(p);
    return hipSuccess;
}

hipError_t hipHostMalloc(void** p, size_t bytes, unsigned)
{
    *p = std::malloc(bytes ? bytes : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t hipHostFree(void* p)
{
    std::free(p);
    return hipSuccess;
}

// ------------------------------------------------------------------------------------------
// Streams, events and graphs.  Work runs at submission unless the stream is capturing: then it
// is appended to the graph being captured.  A stream that waits on an event recorded during a
// capture joins that capture (as HIP's cross-stream capture does); hipStreamEndCapture on the
// origin stream ends it for every joined stream.
// ------------------------------------------------------------------------------------------
struct ihipGraph {
    std::vector<std::function<void()>> nodes;
    hipStream_t origin = nullptr;
};
struct hipGraphExec {
    std::vector<std::function<void()>> nodes;
};
struct ihipStream_t {
    ihipGraph* capturing = nullptr;
};
struct ihipEvent_t {
    bool timing = true;
    bool recorded = false;
    double t = 0;
    ihipGraph* in_capture = nullptr;
};

static double g_clock = 0;             // fake device time in ms: each launch takes 1 us
static std::set<hipStream_t> g_streams;
static std::set<hipEvent_t> g_events;

static hipError_t submit(hipStream_t s, std::function<void()> f)
{
    if (s && !g_streams.count(s)) { fake_error("work submitted to a destroyed stream"); return hipErrorInvalidHandle; }
    if (s && s->capturing) {
        s->capturing->nodes.push_back(std::move(f));
        return hipSuccess;
    }
    f();
    g_clock += 1e-3;
    return hipSuccess;
}

static bool capturing(hipStream_t s) { return s && s->capturing; }

hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind)
{
    if (kind == hipMemcpyDeviceToHost || kind == hipMemcpyDeviceToDevice) touch_read(src, bytes, "hipMemcpy src");
    if (kind == hipMemcpyHostToDevice || kind == hipMemcpyDeviceToDevice) touch_write(dst, bytes, "hipMemcpy dst");
    if (bytes) std::memmove(dst, src, bytes);
    return hipSuccess;
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s)
{
    return submit(s, [=] { (void)hipMemcpy(dst, src, bytes, kind); });
}

hipError_t hipMemsetAsync(void* dst, int value, size_t bytes, hipStream_t s)
{
    return submit(s, [=] {
        touch_write(dst, bytes, "hipMemsetAsync");
        if (bytes) std::memset(dst, value, bytes);
    });
}

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned)
{
    *s = new ihipStream_t();
    g_streams.insert(*s);
    return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s)
{
    if (!g_streams.count(s)) { fake_error("hipStreamDestroy of an unknown stream"); return hipErrorInvalidHandle; }
    if (s->capturing) fake_error("hipStreamDestroy of a stream that is capturing");
    g_streams.erase(s);
    delete s;
    return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s)
{
    if (s && !g_streams.count(s)) { fake_error("hipStreamSynchronize of an unknown stream"); return hipErrorInvalidHandle; }
    if (capturing(s)) { fake_error("hipStreamSynchronize during a capture"); return hipErrorStreamCaptureUnsupported; }
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e)
{
    *e = new ihipEvent_t();
    g_events.insert(*e);
    return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags)
{
    *e = new ihipEvent_t();
    (*e)->timing = !(flags & hipEventDisableTiming);
    g_events.insert(*e);
    return hipSuccess;
}

hipError_t hipEventDestroy(hipEvent_t e)
{
    if (!g_events.count(e)) { fake_error("hipEventDestroy of an unknown event"); return hipErrorInvalidHandle; }
    g_events.erase(e);
    delete e;
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    if (!g_events.count(e)) { fake_error("hipEventRecord of an unknown event"); return hipErrorInvalidHandle; }
    if (s && !g_streams.count(s)) { fake_error("hipEventRecord on a destroyed stream"); return hipErrorInvalidHandle; }
    if (capturing(s)) {
        e->in_capture = s->capturing;
        return hipSuccess;
    }
    e->in_capture = nullptr;
    e->recorded = true;
    e->t = g_clock;
    return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned)
{
    if (!g_events.count(e)) { fake_error("hipStreamWaitEvent on an unknown event"); return hipErrorInvalidHandle; }
    if (s && !g_streams.count(s)) { fake_error("hipStreamWaitEvent on a destroyed stream"); return hipErrorInvalidHandle; }
    if (e->in_capture && s && !s->capturing) s->capturing = e->in_capture;   // joins the capture
    return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t e)
{
    if (!g_events.count(e)) { fake_error("hipEventSynchronize of an unknown event"); return hipErrorInvalidHandle; }
    return hipSuccess;
}

hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b)
{
    if (!g_events.count(a) || !g_events.count(b)) { fake_error("hipEventElapsedTime of an unknown event"); return hipErrorInvalidHandle; }
    if (!a->timing || !b->timing) return hipErrorInvalidHandle;
    if (!a->recorded || !b->recorded) { fake_error("hipEventElapsedTime of an event never recorded"); return hipErrorNotReady; }
    *ms = (float)(b->t - a->t) + 1e-3f;
    return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode)
{
    if (!s) { fake_error("capture on the null stream"); return hipErrorStreamCaptureUnsupported; }
    if (!g_streams.count(s)) { fake_error("capture on an unknown stream"); return hipErrorInvalidHandle; }
    if (s->capturing) { fake_error("nested capture"); return hipErrorIllegalState; }
    s->capturing = new ihipGraph();
    s->capturing->origin = s;
    return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g)
{
    if (!s || !s->capturing || s->capturing->origin != s) { fake_error("hipStreamEndCapture without a capture"); return hipErrorIllegalState; }
    ihipGraph* G = s->capturing;
    for (hipStream_t o : g_streams)
        if (o->capturing == G) o->capturing = nullptr;
    for (hipEvent_t e : g_events)
        if (e->in_capture == G) e->in_capture = nullptr;
    *g = G;
    return hipSuccess;
}

static std::set<hipGraph_t> g_graphs;
static std::set<hipGraphExec_t> g_execs;

hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t g, hipGraphNode_t*, char*, size_t)
{
    *exec = new hipGraphExec();
    (*exec)->nodes = g->nodes;
    g_graphs.insert(g);
    g_execs.insert(*exec);
    return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s)
{
    if (!g_execs.count(exec)) { fake_error("hipGraphLaunch of an unknown executable graph"); return hipErrorInvalidHandle; }
    ++g_fake_graph_launches;
    for (auto& f : exec->nodes) {
        const hipError_t e = submit(s, f);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t exec)
{
    if (!g_execs.count(exec)) { fake_error("hipGraphExecDestroy of an unknown executable graph"); return hipErrorInvalidHandle; }
    g_execs.erase(exec);
    delete exec;
    return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g)
{
    g_graphs.erase(g);
    delete g;
    return hipSuccess;
}

hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int)
{
    std::memset(p, 0, sizeof(*p));
    std::strcpy(p->name, "host stand-in");
    std::strcpy(p->gcnArchName, "gfx950:sramecc+:xnack-");
    p->multiProcessorCount = 256;
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int)
{
    if (a != hipDeviceAttributeMultiprocessorCount) return hipErrorInvalidValue;
    *v = 256;
    return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "stand-in error"; }

extern "C" int fake_live_device_allocations(void) { return (int)g_dev.size(); }
extern "C" int fake_live_streams(void) { return (int)g_streams.size(); }
extern "C" int fake_live_events(void) { return (int)g_events.size(); }

// ------------------------------------------------------------------------------------------
// Launch layer
// ------------------------------------------------------------------------------------------
namespace dk {

bool level_supported(int nf) { return nf == 4 || nf == 8 || nf == 16 || nf == 32 || nf == 64 || nf == 128; }

int shape_rows(int nf, int v)
{
    switch (nf) {
        case 4: return v == 0 ? 4 : 0;
        case 8: { const int r[] = {8, 2, 4, 8}; return v >= 0 && v < 4 ? r[v] : 0; }
        case 16: { const int r[] = {8, 4, 2, 8}; return v >= 0 && v < 4 ? r[v] : 0; }
        case 32: { const int r[] = {8, 4, 16, 8}; return v >= 0 && v < 4 ? r[v] : 0; }
        case 64: { const int r[] = {8, 16, 8}; return v >= 0 && v < 3 ? r[v] : 0; }
        case 128: { const int r[] = {8, 16}; return v >= 0 && v < 2 ? r[v] : 0; }
        default: return 0;
    }
}

int shape_spw(int nf, int v)
{
    const int r = shape_rows(nf, v);
    if (r == 0) return 0;
    const int ts = (nf / 2) * (nf / r);
    const int base = ts >= 256 ? 1 : 256 / ts;
    const bool wide = (nf == 8 || nf == 16 || nf == 32) ? v == 3 : (nf == 64 ? v == 2 : false);
    return wide ? 4 * base : base;
}

static void level_tables(const LevelArgs& A, bool pair, size_t esize, const char* who)
{
    const size_t nn = (size_t)A.nf * A.nf, nc = nn / 4;
    touch_read(A.rho0_f, esize * nn, who);
    touch_read(A.phi_f, sizeof(double) * A.n_obs * nn, who);
    touch_read(A.obs_f, sizeof(double) * 3 * A.n_obs, who);
    if (pair) {
        touch_read(A.rho0_c, esize * nc, who);
        touch_read(A.phi_c, sizeof(double) * A.n_obs * nc, who);
        touch_read(A.obs_c, sizeof(double) * 3 * A.n_obs, who);
    }
}

hipError_t launch_level(const LevelKind& k, const LevelArgs& A, hipStream_t s)
{
    if (!level_supported(A.nf)) return hipErrorInvalidValue;
    if (k.noise && k.precision == DK_PREC_F32 && shape_rows(A.nf, k.shape) == 0) return hipErrorInvalidValue;
    if (A.count == 0) return hipSuccess;
    ++g_fake_launches;
    const LevelArgs a = A;
    const LevelKind kk = k;
    return submit(s, [a, kk] {
        const size_t esize = (!kk.noise || kk.precision == DK_PREC_F64) ? 8 : 4;
        const size_t nn = (size_t)a.nf * a.nf;
        level_tables(a, kk.pair, esize, "launch_level tables");
        const int nobs = a.n_obs;
        touch_write(a.out, sizeof(double) * 2 * nobs * a.count, "launch_level out");
        if (a.field_f) touch_write(a.field_f, esize * nn * a.count, "launch_level field_f");
        if (a.field_c) touch_write(a.field_c, esize * nn / 4 * a.count, "launch_level field_c");
        if (!kk.noise) {
            for (int j = 0; j < nobs; ++j) {
                a.out[2 * j] = 0.25 + 0.01 * j;
                a.out[2 * j + 1] = 0.0;
            }
            return;
        }
        for (uint64_t i = 0; i < a.count; ++i)
            for (int j = 0; j < nobs; ++j) {
                a.out[(i * nobs + j) * 2 + 0] = fake_value(a.seed, a.tag, a.level_id, a.first + i, j, kk.pair, 0);
                a.out[(i * nobs + j) * 2 + 1] = fake_value(a.seed, a.tag, a.level_id, a.first + i, j, kk.pair, 1);
            }
    });
}

static void neumaier(double& s, double& c, double x)
{
    const double t = s + x;
    if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

static void moments_of(const double* ps, uint64_t count, int nobs, double* out /* [nobs][6][2] */)
{
    for (int j = 0; j < nobs; ++j)
        for (int k = 0; k < DK_NMOM; ++k) {
            double s = 0, c = 0;
            for (uint64_t i = 0; i < count; ++i) {
                const double pf = ps[(i * nobs + j) * 2], pc = ps[(i * nobs + j) * 2 + 1], y = pf - pc;
                const double v = k == 0 ? y : k == 1 ? y * y : k == 2 ? pf : k == 3 ? pf * pf : k == 4 ? pc : pc * pc;
                neumaier(s, c, v);
            }
            out[(j * DK_NMOM + k) * 2] = s;
            out[(j * DK_NMOM + k) * 2 + 1] = c;
        }
}

hipError_t launch_moments(const double* per_sample, uint64_t count, int n_obs, double* out, hipStream_t s)
{
    ++g_fake_launches;
    return submit(s, [=] {
        touch_read(per_sample, sizeof(double) * 2 * n_obs * count, "launch_moments in");
        touch_write(out, sizeof(double) * 2 * DK_NMOM * n_obs, "launch_moments out");
        moments_of(per_sample, count, n_obs, out);
    });
}

hipError_t launch_field_eval(const FieldDev&, double, int n, void* out, bool as_double, hipStream_t s)
{
    ++g_fake_launches;
    return submit(s, [=] {
        const size_t nn = (size_t)n * n;
        touch_write(out, (as_double ? 8 : 4) * nn, "launch_field_eval");
        for (size_t i = 0; i < nn; ++i) {
            if (as_double) ((double*)out)[i] = 1.0;
            else ((float*)out)[i] = 1.0f;
        }
    });
}

hipError_t launch_noise_dump(uint64_t, uint32_t, int, int n, uint64_t, uint32_t n_samples, int, int n_steps, float* out,
                             hipStream_t s)
{
    return submit(s, [=] { touch_write(out, sizeof(float) * 2 * (size_t)n * n * n_steps * n_samples, "launch_noise_dump"); });
}

hipError_t launch_gauss(const uint32_t* a, const uint32_t* b, uint64_t count, float* z0, float* z1, hipStream_t s)
{
    return submit(s, [=] {
        touch_read(a, 4 * count, "launch_gauss a");
        touch_read(b, 4 * count, "launch_gauss b");
        touch_write(z0, 4 * count, "launch_gauss z0");
        touch_write(z1, 4 * count, "launch_gauss z1");
    });
}

hipError_t launch_meanfield_stream(int n, double, int steps, double* buf0, double* buf1, double** result, hipStream_t s)
{
    double* in = buf0;
    double* out = buf1;
    for (int m = 0; m < steps; ++m) {
        const hipError_t e = submit(s, [=] {
            touch_read(in, sizeof(double) * n * n, "meanfield in");
            touch_write(out, sizeof(double) * n * n, "meanfield out");
        });
        if (e != hipSuccess) return e;
        std::swap(in, out);
    }
    *result = in;
    return hipSuccess;
}

hipError_t launch_inner_products(const double* rho, int n, const double* phi, int n_obs, double, double* out, hipStream_t s)
{
    return submit(s, [=] {
        touch_read(rho, sizeof(double) * n * n, "inner rho");
        touch_read(phi, sizeof(double) * n_obs * n * n, "inner phi");
        touch_write(out, sizeof(double) * n_obs, "inner out");
        for (int j = 0; j < n_obs; ++j) out[j] = 0.25 + 0.01 * j;
    });
}

// ---- persistent round kernel ----
int round_kind(int nf, bool pair)
{
    switch (nf) {
        case 8: return pair ? -1 : 0;
        case 16: return pair ? 5 : 1;
        case 32: return pair ? 6 : 2;
        case 64: return pair ? 7 : 3;
        case 128: return pair ? 8 : 4;
        default: return -1;
    }
}
int round_spw_of(int nf)
{
    switch (nf) {
        case 8: return 256; case 16: return 64; case 32: return 16; case 64: return 4; case 128: return 1;
        default: return 0;
    }
}
int round_blocks_per_cu(int) { return 1; }
int round_max_obs() { return 1024 / DK_NMOM; }

hipError_t launch_round(const RoundArgs& P, int, int grid, hipStream_t s)
{
    if (grid <= 0 || P.n_obs <= 0 || P.n_obs * DK_NMOM > 1024) return hipErrorInvalidValue;
    ++g_fake_launches;
    const RoundArgs a = P;
    return submit(s, [a, grid] {
        touch_read(a.ntasks, sizeof(uint32_t), "round ntasks");
        touch_write(a.head, sizeof(uint32_t), "round head");
        touch_write(a.scratch, sizeof(double) * a.scratch_stride * grid, "round scratch");
        const uint32_t nt = *a.ntasks;
        touch_read(a.tasks, sizeof(RoundTask) * nt, "round tasks");
        const int nobs = a.n_obs;
        touch_write(a.task_mom, sizeof(double) * 2 * DK_NMOM * nobs * nt, "round task moments");
        for (uint32_t t = 0; t < nt; ++t) {
            const RoundTask T = a.tasks[t];
            if (T.level >= (uint32_t)DK_MAX_LEVELS) { fake_error("round task %u: level %u", t, T.level); continue; }
            touch_read(a.levels + T.level, sizeof(RoundLevel), "round level");
            const RoundLevel L = a.levels[T.level];
            const bool pair = L.kind >= 5;
            if (L.kind != round_kind(L.A.nf, pair) || L.kind < 0)
                fake_error("round task %u: kind %d does not match n = %d", t, L.kind, L.A.nf);
            if (L.spw != round_spw_of(L.A.nf)) fake_error("round task %u: spw %d for n = %d", t, L.spw, L.A.nf);
            level_tables(L.A, pair, 4, "round level tables");
            std::vector<double> ps((size_t)2 * nobs * T.count);
            for (uint64_t i = 0; i < T.count; ++i)
                for (int j = 0; j < nobs; ++j) {
                    ps[(i * nobs + j) * 2] = fake_value(L.A.seed, L.A.tag, L.A.level_id, T.first + i, j, pair, 0);
                    ps[(i * nobs + j) * 2 + 1] = fake_value(L.A.seed, L.A.tag, L.A.level_id, T.first + i, j, pair, 1);
                }
            moments_of(ps.data(), T.count, nobs, a.task_mom + (size_t)t * nobs * DK_NMOM * 2);
        }
    });
}

// ---- streaming kernels: state words 0..4 of each sample hold (sample, level, tag, seed, step) ----
bool stream_supported(int nf) { return nf >= 64 && nf % 64 == 0; }
bool stream_depth_supported(int depth) { return depth == 1 || depth == 2 || depth == 4 || depth == 8; }

static const uint32_t kUnset = 0xFFFFFFFFu;

static void put_id(float* st, uint64_t sample, int level, uint32_t tag, uint64_t seed, uint32_t step)
{
    const uint32_t w[5] = {(uint32_t)sample, (uint32_t)level, tag, (uint32_t)seed, step};
    std::memcpy(st, w, sizeof(w));
}

static void get_id(const float* st, uint32_t w[5]) { std::memcpy(w, st, 5 * sizeof(uint32_t)); }

hipError_t launch_stream_init(const float* rho0, int n, int count, float* rho, float* cmp, hipStream_t s)
{
    ++g_fake_launches;
    return submit(s, [=] {
        const size_t nn = (size_t)n * n;
        touch_read(rho0, 4 * nn, "stream_init rho0");
        touch_write(rho, 4 * nn * count, "stream_init rho");
        touch_write(cmp, 4 * nn * count, "stream_init cmp");
        for (int i = 0; i < count; ++i) {
            const uint32_t w[5] = {kUnset, kUnset, kUnset, kUnset, 0};
            std::memcpy(rho + i * nn, w, sizeof(w));
        }
    });
}

static void advance(const float* in, float* out, size_t per, int count, uint64_t first, int level, uint32_t tag,
                    uint64_t seed, uint32_t from, uint32_t to, const char* who)
{
    for (int i = 0; i < count; ++i) {
        uint32_t w[5];
        get_id(in + i * per, w);
        if (w[4] != from) fake_error("%s: sample %llu is at step %u, the launch starts at %u", who,
                                     (unsigned long long)(first + i), w[4], from);
        if (w[0] != kUnset && (w[0] != (uint32_t)(first + i) || w[1] != (uint32_t)level || w[2] != tag || w[3] != (uint32_t)seed))
            fake_error("%s: slot %d holds sample %u (level %u), the launch advances sample %llu (level %d)", who, i, w[0], w[1],
                       (unsigned long long)(first + i), level);
        put_id(out + i * per, first + i, level, tag, seed, to);
    }
}

hipError_t launch_stream_step(const StreamArgs& A, bool pair, int, int depth, hipStream_t s)
{
    if (A.ksteps < 1 || A.ksteps > depth || (pair && depth != 4 && !A.z)) return hipErrorInvalidValue;
    if (!stream_depth_supported(depth)) return hipErrorInvalidValue;
    ++g_fake_launches;
    const StreamArgs a = A;
    return submit(s, [a, pair, depth] {
        const size_t nn = (size_t)a.n * a.n, nc = nn / 4;
        touch_read(a.rho_in, 4 * nn * a.count, "stream_step rho_in");
        touch_read(a.cmp_in, 4 * nn * a.count, "stream_step cmp_in");
        touch_write(a.rho_out, 4 * nn * a.count, "stream_step rho_out");
        touch_write(a.cmp_out, 4 * nn * a.count, "stream_step cmp_out");
        if (a.rho_in == a.rho_out) fake_error("stream_step: input and output state are one buffer");
        advance(a.rho_in, a.rho_out, nn, a.count, a.first, a.level_id, a.tag, a.seed, (uint32_t)a.m0,
                (uint32_t)(a.m0 + a.ksteps), "stream_step fine");
        if (!pair) return;
        if (depth == 4) {
            if ((a.m0 % 4) != 0 || !a.do_coarse) fake_error("stream_step: depth-4 pair launch at step %d, do_coarse %d", a.m0, a.do_coarse);
            touch_read(a.rhoc_in, 4 * nc * a.count, "stream_step rhoc_in");
            touch_read(a.cmpc_in, 4 * nc * a.count, "stream_step cmpc_in");
            touch_write(a.rhoc_out, 4 * nc * a.count, "stream_step rhoc_out");
            touch_write(a.cmpc_out, 4 * nc * a.count, "stream_step cmpc_out");
            advance(a.rhoc_in, a.rhoc_out, nc, a.count, a.first, a.level_id, a.tag, a.seed, (uint32_t)(a.m0 / 4),
                    (uint32_t)(a.m0 / 4 + 1), "stream_step coarse");
            return;
        }
        // split groups: running sums of the group that the launch continues, stored at its end;
        // words 0..4 of each sample's slot hold (sample, level, tag, seed, group index)
        if (a.zgroup < nc * a.count) fake_error("stream_step: zgroup too small");
        const int groups = depth == 8 ? a.ksteps / 4 : 1;
        if (depth == 8 && (a.ksteps % 4) != 0) fake_error("stream_step: depth-8 pair launch of %d steps", a.ksteps);
        if (a.z_load) {
            touch_read(a.z, 8 * nc * a.count, "stream_step z load");
            for (int i = 0; i < a.count; ++i) {
                uint32_t w[5];
                get_id(a.z + 2 * (size_t)i * nc, w);
                if (w[0] != (uint32_t)(a.first + i) || w[1] != (uint32_t)a.level_id || w[4] != (uint32_t)(a.m0 / 4))
                    fake_error("stream_step: restricted sums of slot %d hold sample %u group %u, the launch continues "
                               "sample %llu group %d", i, w[0], w[4], (unsigned long long)(a.first + i), a.m0 / 4);
            }
        }
        for (int g = 0; g < groups; ++g) {
            float* zg = a.z + 2 * g * a.zgroup;
            touch_write(zg, 8 * nc * a.count, "stream_step z store");
            for (int i = 0; i < a.count; ++i)
                put_id(zg + 2 * (size_t)i * nc, a.first + i, a.level_id, a.tag, a.seed, (uint32_t)(a.m0 / 4 + g));
        }
    });
}

hipError_t launch_stream_coarse(int nc, int count, float, float, int, const float* rho_in, const float* cmp_in, const float* z,
                                float* rho_out, float* cmp_out, hipStream_t s)
{
    ++g_fake_launches;
    return submit(s, [=] {
        const size_t cc = (size_t)nc * nc;
        touch_read(rho_in, 4 * cc * count, "stream_coarse rho_in");
        touch_read(cmp_in, 4 * cc * count, "stream_coarse cmp_in");
        touch_read(z, 8 * cc * count, "stream_coarse z");
        touch_write(rho_out, 4 * cc * count, "stream_coarse rho_out");
        touch_write(cmp_out, 4 * cc * count, "stream_coarse cmp_out");
        for (int i = 0; i < count; ++i) {
            uint32_t w[5], zw[5];
            get_id(rho_in + i * cc, w);
            get_id(z + 2 * (size_t)i * cc, zw);
            if (w[4] != zw[4]) fake_error("stream_coarse: slot %d is at coarse step %u, its noise sums are of group %u", i, w[4], zw[4]);
            if (w[0] != kUnset && (w[0] != zw[0] || w[1] != zw[1] || w[2] != zw[2] || w[3] != zw[3]))
                fake_error("stream_coarse: slot %d holds sample %u, its noise sums are of sample %u", i, w[0], zw[0]);
            zw[4] += 1;
            std::memcpy(rho_out + i * cc, zw, sizeof(zw));
        }
    });
}

hipError_t launch_stream_copy(const float* a, const float* b, size_t total, float* a2, float* b2, hipStream_t s)
{
    return submit(s, [=] {
        touch_read(a, 4 * total, "stream_copy a");
        touch_read(b, 4 * total, "stream_copy b");
        touch_write(a2, 4 * total, "stream_copy a2");
        touch_write(b2, 4 * total, "stream_copy b2");
    });
}

hipError_t launch_stream_observe(const float* rho, int n, int count, const double* phi, const double* obs, int n_obs,
                                 double, double* out, int slot, hipStream_t s)
{
    ++g_fake_launches;
    return submit(s, [=] {
        const size_t nn = (size_t)n * n;
        touch_read(rho, 4 * nn * count, "stream_observe rho");
        touch_read(phi, sizeof(double) * n_obs * nn, "stream_observe phi");
        touch_read(obs, sizeof(double) * 3 * n_obs, "stream_observe obs");
        touch_write(out, sizeof(double) * 2 * n_obs * count, "stream_observe out");
        for (int i = 0; i < count; ++i) {
            uint32_t w[5];
            get_id(rho + i * nn, w);
            if (w[0] == kUnset) { fake_error("stream_observe: sample slot %d was never advanced", i); continue; }
            // the coarse state of a pair carries the fine level's identity
            for (int j = 0; j < n_obs; ++j)
                out[((size_t)i * n_obs + j) * 2 + slot] = fake_value(w[3], w[2], (int)w[1], w[0], j, slot == 1, slot);
        }
    });
}

hipError_t launch_zero_slot(double* out, int count, int n_obs, int slot, hipStream_t s)
{
    if (count * n_obs <= 0) return hipSuccess;
    return submit(s, [=] {
        touch_write(out, sizeof(double) * 2 * n_obs * count, "zero_slot out");
        for (int i = 0; i < count * n_obs; ++i) out[(size_t)i * 2 + slot] = 0.0;
    });
}

hipError_t launch_heat_f32(const float* in, float* out, int n, int batch, float, hipStream_t s)
{
    return submit(s, [=] {
        touch_read(in, 4 * (size_t)n * n * batch, "heat in");
        touch_write(out, 4 * (size_t)n * n * batch, "heat out");
    });
}

// ---- couplings and schemes the harness does not drive ----
bool fourier_supported(int, bool) { return false; }
int fourier_grid(int, int, uint64_t) { return 1; }
size_t fourier_scratch_elems(int) { return 0; }
hipError_t launch_fourier(const FourierArgs&, int, bool, int, hipStream_t) { return hipErrorInvalidValue; }
bool theta_supported(int, bool) { return false; }
int theta_grid(int, int, uint64_t) { return 1; }
hipError_t launch_theta(const ThetaArgs&, int, bool, int, hipStream_t) { return hipErrorInvalidValue; }

namespace cnn {
hipError_t Workspace::reserve(int, int) { return hipErrorInvalidValue; }
void Workspace::release() {}
hipError_t pack(Workspace&, const float*, hipStream_t) { return hipErrorInvalidValue; }
hipError_t forward(Workspace&, const float*, const float*, int, float*, hipStream_t) { return hipErrorInvalidValue; }
hipError_t backward(Workspace&, const float*, const float*, const float*, const float*, int, float*, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t adam_update(float*, const float*, float*, float*, float, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t normalize(const void*, bool, const double*, int, size_t, double, float*, hipStream_t) { return hipErrorInvalidValue; }
hipError_t extract_y(const double*, int, int, int, float*, hipStream_t) { return hipErrorInvalidValue; }
hipError_t combine_cv(const double*, int, int, const float*, const float*, int, int, double*, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t accumulate_sq(const Workspace&, int, double*, hipStream_t) { return hipErrorInvalidValue; }
}  // namespace cnn

}  // namespace dk

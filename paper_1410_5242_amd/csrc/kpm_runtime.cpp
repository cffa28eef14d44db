// Host runtime behind the C ABI (include/kpm.h): argument validation, device
// allocations, workspace caching and the launch sequence of the KPM
// iteration.  No arithmetic of the method runs here beyond the two-number
// scaling (a, b) from the Gershgorin bounds; everything else is enqueued as
// device kernels on the caller's stream.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "kpm_internal.h"

namespace kpm {

namespace {
thread_local std::string g_error;

// Scalar-product partials of this many consecutive sweeps are kept on the
// device before one reduction launch folds them into eta.
constexpr int kReduceEvery = 64;

bool r_supported(int R) {
    return R == 1 || R == 2 || R == 4 || R == 8 || R == 16 || R == 32 || R == 64;
}

size_t real_size(int dtype) { return dtype == KPM_C128 ? sizeof(double) : sizeof(float); }

kpm_status fail(kpm_status st, const std::string& msg) {
    set_error(msg);
    return st;
}

kpm_status hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? KPM_ENOMEM : KPM_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define KPM_HIP(call, what)                           \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

kpm_status check_device(const kpm_hamiltonian* H) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(KPM_EDEVICE, "hipGetDevice failed");
    if (dev != H->device) return fail(KPM_EINVAL, "current device differs from the device H was built on");
    return KPM_OK;
}

bool use_lattice(const kpm_hamiltonian* H, int R);

// Column-group width kpm_moments takes by default.  On a lattice the
// lattice sweep runs 32 columns at a time: for R = 64 two 32-column
// recurrences beat one recurrence whose sweeps take both halves (64^3 and
// 128 x 128 x 64, both precisions: 3.5-3.8 % faster; 96 x 96 x 64: 15 %),
// so the block is split when the caller wants no raw eta of the whole
// block (split = true).  Otherwise the whole block where it fits the
// sweeps' 32-bit buffer offsets (the padding row of imported matrices
// included), else the widest supported width that does, except that the
// groups stop at 32 columns where the lattice sweep runs there: it then
// addresses its arrays plane by plane (128^3 sites at R = 32 in complex128:
// 2.69 ms per sweep against 3.75 ms as 16-column groups on the window
// sweep).
int default_group(const kpm_hamiltonian* H, int R, bool split) {
    const uint64_t lim = (1ull << 32) - (1ull << 24);
    auto fits = [&](int g) { return (static_cast<uint64_t>(H->nrows) + 1) * g * 2 * real_size(H->dtype) < lim; };
    int G = R;
    if (split && R > 32 && use_lattice(H, 32)) G = 32;
    while (G > 1 && !fits(G) && !(G == 32 && use_lattice(H, 32))) G /= 2;
    return G;
}

// The SELL-C-sigma sweep addresses a block with 32-bit offsets, the padding
// column N included.
kpm_status check_sell_block(const kpm_hamiltonian* H, int R) {
    if (H->sell.C == 0) return KPM_OK;
    const uint64_t bytes = (static_cast<uint64_t>(H->nrows) + 1) * R * 2 * real_size(H->dtype);
    if (bytes >= (1ull << 32) - 64) return fail(KPM_ENOTSUP, "an [N+1][R] block over SELL storage reaches 4 GiB");
    return KPM_OK;
}

template <typename P>
kpm_status grow(P** ptr, size_t* have, size_t need, const char* what) {
    if (*have >= need && *ptr) return KPM_OK;
    if (*ptr) {
        KPM_HIP(hipFree(*ptr), "hipFree");
        *ptr = nullptr;
        *have = 0;
    }
    void* p = nullptr;
    KPM_HIP(hipMalloc(&p, need), what);
    *ptr = static_cast<P*>(p);
    *have = need;
    return KPM_OK;
}

// The workspace of H for the calls on stream s (created on first use).
Workspace* workspace(kpm_hamiltonian* H, hipStream_t s) {
    std::lock_guard<std::mutex> g(H->lock);
    auto it = H->ws.find(s);
    if (it != H->ws.end()) return it->second;
    Workspace* w = new Workspace();
    H->ws.emplace(s, w);
    return w;
}

kpm_status ensure_vectors(Workspace& w, const kpm_hamiltonian* H, int R) {
    const size_t need = static_cast<size_t>(H->nrows) * 2 * R * real_size(H->dtype);
    for (int i = 0; i < 2; ++i) {
        size_t have = w.vbytes;
        kpm_status st = grow(&w.vbuf[i], &have, need, "hipMalloc(vector block)");
        if (st != KPM_OK) return st;
    }
    if (w.vbytes < need) w.vbytes = need;
    return KPM_OK;
}

// Grid of the sweep kernel that kpm_moments / kpm_aug_spmmv will launch.
// The lattice kernel runs one workgroup per 4 x 4-site pencil; below about
// half a workgroup per CU the generic sweep fills the machine better.
bool use_lattice(const kpm_hamiltonian* H, int R) {
    const int t = get_tuning().lattice;
    if (t == 0 || !lattice_supported(H, R)) return false;
    return t == 2 || lattice_tiles(H) >= 128;
}

// The per-die tile counters are read only by the scalar-operand sweep with
// dynamic tile mapping; the other sweeps need no cleared queue.
bool sweep_uses_queue(const kpm_hamiltonian* H, int R) {
    return H->sell.C == 0 && !use_lattice(H, R) && !use_gather(H->dtype, R, H->nrows) && get_tuning().dynamic != 0;
}

// The LDS-window variant of the staged-gather sweep (tuning gather 1:
// where it exists and the lattice gives at least one run of z-planes of a
// tile per CU; 3: wherever it exists).
bool use_window(const kpm_hamiltonian* H, int R) {
    const int g = get_tuning().gather;
    if ((g != 1 && g != 3) || use_lattice(H, R) || !use_gather(H->dtype, R, H->nrows)) return false;
    const int side = gather_window_side(H->dtype, R);
    if (side <= 0 || H->L[0] <= 0) return false;
    if (g == 3) return true;
    const int64_t ntiles = static_cast<int64_t>((H->L[0] + side - 1) / side) * ((H->L[1] + side - 1) / side);
    const int64_t cus = device_cus();
    const int64_t cap = H->L[2] >= 8 ? H->L[2] / 4 : 1;
    int64_t np = (cus + ntiles - 1) / ntiles;
    np = np < 1 ? 1 : (np > cap ? cap : np);
    return ntiles * np >= cus;
}

int launch_grid(const kpm_hamiltonian* H, int R) {
    if (H->sell.C > 0) return sell_grid(H->dtype, R, H->nrows);
    return use_lattice(H, R) ? lattice_grid(H) : sweep_grid(H->dtype, R, H->nrows, use_window(H, R));
}

// Sweep kernel kind (kpm_sweep_kernel): 1 lattice, 3 window, 2 staged
// gather, 0 scalar operand, 4 SELL-C-sigma.
int sweep_kind(const kpm_hamiltonian* H, int R) {
    if (H->sell.C > 0) return 4;
    if (use_lattice(H, R)) return 1;
    if (!use_gather(H->dtype, R, H->nrows)) return 0;
    return use_window(H, R) ? 3 : 2;
}

kpm_status ensure_partials(Workspace& w, const kpm_hamiltonian* H, int R, int slots) {
    const int grid = launch_grid(H, R);
    const size_t need = static_cast<size_t>(slots) * grid * 3 * R * sizeof(double);
    return grow(&w.partials, &w.pbytes, need, "hipMalloc(partials)");
}

// Sites in processing order: pencils of P x P sites over the full z extent,
// pencils ordered x-block fastest, each pencil walked plane by plane with x
// fastest.  Every site appears exactly once.
std::vector<int32_t> pencil_schedule(const int L[3], int P) {
    std::vector<int32_t> s;
    s.reserve(static_cast<size_t>(L[0]) * L[1] * L[2]);
    for (int by = 0; by < L[1]; by += P)
        for (int bx = 0; bx < L[0]; bx += P)
            for (int z = 0; z < L[2]; ++z)
                for (int y = by; y < by + P && y < L[1]; ++y)
                    for (int x = bx; x < bx + P && x < L[0]; ++x)
                        s.push_back(static_cast<int32_t>(x + static_cast<int64_t>(L[0]) * (y + static_cast<int64_t>(L[1]) * z)));
    return s;
}

// H's site schedule for the current tuning's pencil side (nullptr: natural
// order); schedules are built once per side and kept until H is destroyed.
kpm_status schedule_for(kpm_hamiltonian* H, const int32_t** out) {
    *out = nullptr;
    const int P = get_tuning().pencil;
    if (P <= 0 || H->sell.C > 0) return KPM_OK;
    std::lock_guard<std::mutex> g(H->lock);
    auto it = H->sched.find(P);
    if (it != H->sched.end()) {
        *out = it->second;
        return KPM_OK;
    }
    std::vector<int32_t> s = pencil_schedule(H->L, P);
    if (static_cast<int64_t>(s.size()) * 4 != H->nrows) return fail(KPM_EINTERNAL, "schedule size mismatch");
    int32_t* d = nullptr;
    KPM_HIP(hipMalloc(&d, s.size() * sizeof(int32_t)), "hipMalloc(schedule)");
    const hipError_t e = hipMemcpy(d, s.data(), s.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(e, "copy schedule");
    }
    H->sched.emplace(P, d);
    *out = d;
    return KPM_OK;
}

kpm_status ensure_queue(Workspace& w) {
    return grow(&w.queue, &w.qbytes, static_cast<size_t>(kReduceEvery) * kXcds * sizeof(int), "hipMalloc(queue)");
}

kpm_status ensure_flag(Workspace& w) {
    if (!w.flag) KPM_HIP(hipMalloc(&w.flag, sizeof(int)), "hipMalloc(flag)");
    if (!w.flag_host) KPM_HIP(hipHostMalloc(&w.flag_host, sizeof(int)), "hipHostMalloc(flag)");
    return KPM_OK;
}

void free_workspace(Workspace* w) {
    if (!w) return;
    for (int i = 0; i < 2; ++i)
        if (w->vbuf[i]) (void)hipFree(w->vbuf[i]);
    if (w->partials) (void)hipFree(w->partials);
    if (w->queue) (void)hipFree(w->queue);
    if (w->eta) (void)hipFree(w->eta);
    if (w->mu) (void)hipFree(w->mu);
    if (w->flag) (void)hipFree(w->flag);
    if (w->flag_host) (void)hipHostFree(w->flag_host);
    for (int i = 0; i < 3; ++i)
        if (w->naive[i]) (void)hipFree(w->naive[i]);
    if (w->dot_part) (void)hipFree(w->dot_part);
    if (w->lanczos) (void)hipFree(w->lanczos);
    if (w->exec) (void)hipGraphExecDestroy(w->exec);
    if (w->graph) (void)hipGraphDestroy(w->graph);
    if (w->capture) (void)hipStreamDestroy(w->capture);
    delete w;
}

// Event pairs around sweep launches (kpm_sweep_profile_*): every period-th
// launch is timed (0: off).  Guarded by `lock`; events are created once and
// reused after each read.
struct SweepProfile {
    std::mutex lock;
    int period = 0;
    uint64_t seen = 0;
    std::vector<hipEvent_t> start, stop;
    size_t used = 0;
};
SweepProfile g_prof;

// Launch through `launch`, bracketed by an event pair when the profile picks
// this launch.  `capturing`: the launch is being recorded into a graph,
// where no events are recorded.
template <class Launch>
hipError_t profiled(hipStream_t s, bool capturing, Launch&& launch) {
    if (capturing) return launch();
    std::unique_lock<std::mutex> g(g_prof.lock);
    if (g_prof.period <= 0 || (g_prof.seen++ % static_cast<uint64_t>(g_prof.period)) != 0) {
        g.unlock();
        return launch();
    }
    if (g_prof.used == g_prof.start.size()) {
        hipEvent_t e0, e1;
        hipError_t e = hipEventCreate(&e0);
        if (e != hipSuccess) return e;
        if ((e = hipEventCreate(&e1)) != hipSuccess) return e;
        g_prof.start.push_back(e0);
        g_prof.stop.push_back(e1);
    }
    const size_t k = g_prof.used++;
    hipError_t e = hipEventRecord(g_prof.start[k], s);
    if (e != hipSuccess) return e;
    if ((e = launch()) != hipSuccess) return e;
    return hipEventRecord(g_prof.stop[k], s);
}

// Tile order the lattice sweep uses: tuning 3 (auto) is round-robin when
// the workgroups take several pencils each, the per-die 2-D blocks otherwise
int lattice_order(const kpm_hamiltonian* H, int grid) {
    const int order = get_tuning().tile_order;
    return order == 3 ? (lattice_tiles(H) > grid ? 2 : 0) : order;
}

// One fused sweep: the cache-blocked lattice kernel where it applies, the
// generic gather kernel otherwise.
hipError_t launch_any_sweep(kpm_hamiltonian* H, int R, int variant, const SweepArgs& a, hipStream_t s,
                            bool capturing = false) {
    if (H->sell.C > 0) {
        const SellStore& c = H->sell;
        SellArgs sa{H->val, H->col, c.start, c.width, c.perm, H->nrows, c.stored, c.clog,
                    a.V, a.W, a.alpha, a.beta, a.gamma, a.partials, a.grid};
        return profiled(s, capturing, [&] { return launch_sell(H->dtype, R, variant, sa, s); });
    }
    if (use_lattice(H, R)) {
        const kpm_sweep_tuning t = get_tuning();
        LatticeArgs la{H->val, a.V, a.W, a.alpha, a.beta, a.gamma, a.partials,
                       {H->L[0], H->L[1], H->L[2]}, {H->periodic[0], H->periodic[1], H->periodic[2]}, a.grid,
                       t.prefetch, t.stream, lattice_order(H, a.grid), R};
        return profiled(s, capturing, [&] { return launch_lattice(H->dtype, variant, la, s); });
    }
    SweepArgs g = a;
    g.window = use_window(H, R) ? 1 : 0;
    return profiled(s, capturing, [&] { return launch_sweep(H->dtype, R, variant, g, s); });
}

// ---- batched solver: launch shape (process-wide) and state per (device, stream) ----
constexpr kpm_batch_tuning kDefaultBatchTuning = {0, 0, 1, 0};
std::mutex g_batch_lock;   // guards g_batch_tuning and the g_batch map (not the states in it)
kpm_batch_tuning g_batch_tuning = kDefaultBatchTuning;

struct BatchState {
    BatchInst* inst = nullptr;          // device instance table
    size_t inst_bytes = 0;
    int32_t* order = nullptr;           // device processing order
    size_t order_bytes = 0;
    int* ints = nullptr;                // device [0] instance counter, [1] spectrum flag
    int* flag_host = nullptr;           // pinned mirror of ints[1]
    void* vec = nullptr;                // two work blocks per instance
    size_t vec_bytes = 0;
    double* eta = nullptr;              // per instance [M/2][3][R]
    size_t eta_bytes = 0;
    hipStream_t capture = nullptr;      // private stream the graph is captured on
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // what the captured graph was made for
    std::vector<BatchInst> key_inst;
    std::vector<int32_t> key_order;
    int key_dtype = -1, key_R = 0, key_M = 0, key_grid = 0, key_waves = 0, key_dynamic = -1, key_slab = -1;
};
// One state per (device, stream): calls on one stream run in order and may
// reuse it.  States are never freed before the process ends, so a pointer
// taken under g_batch_lock stays valid.
std::map<std::pair<int, hipStream_t>, BatchState*> g_batch;

BatchState* batch_state(int dev, hipStream_t s) {
    std::lock_guard<std::mutex> g(g_batch_lock);
    BatchState*& b = g_batch[{dev, s}];
    if (!b) b = new BatchState();
    return b;
}

kpm_batch_tuning batch_tuning() {
    std::lock_guard<std::mutex> g(g_batch_lock);
    return g_batch_tuning;
}

void drop_graph(BatchState& b) {
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
    b.key_inst.clear();
    b.key_order.clear();
}

bool same_inst(const BatchInst& x, const BatchInst& y) {
    return x.val == y.val && x.v0 == y.v0 && x.a == y.a && x.b == y.b && x.eta == y.eta && x.mu == y.mu &&
           x.nrows == y.nrows && x.inv_a == y.inv_a && x.shift == y.shift && x.L[0] == y.L[0] &&
           x.L[1] == y.L[1] && x.L[2] == y.L[2];
}

template <typename X>
void key_add(std::vector<unsigned char>& k, const X& x) {
    const auto* p = reinterpret_cast<const unsigned char*>(&x);
    k.insert(k.end(), p, p + sizeof(X));
}

void drop_moments_graph(Workspace& w) {
    if (w.exec) (void)hipGraphExecDestroy(w.exec);
    if (w.graph) (void)hipGraphDestroy(w.graph);
    w.exec = nullptr;
    w.graph = nullptr;
    w.graph_key.clear();
}

// SELL-C-sigma layout of a CRS pattern (kpm_sell_layout): validation, the
// stable sort by decreasing row length inside windows of sigma rows, chunk
// widths and starts.  len_sorted: row lengths by sorted position.
kpm_status sell_layout(int64_t N, const int64_t* rowptr, int C, int sigma, std::vector<int32_t>& perm,
                       std::vector<int32_t>& width, std::vector<int64_t>& start, std::vector<int32_t>& len_sorted) {
    if (N < 1) return fail(KPM_EINVAL, "N must be >= 1");
    if (N > INT32_MAX - 1) return fail(KPM_ENOMEM, "more than 2^31 - 2 rows");
    if (!rowptr) return fail(KPM_EINVAL, "rowptr is NULL");
    if (C < 1 || C > 64 || (C & (C - 1)) != 0) return fail(KPM_EINVAL, "C must be a power of two in 1..64");
    if (sigma < 1 || (sigma != 1 && sigma % C != 0)) return fail(KPM_EINVAL, "sigma must be 1 or a multiple of C");
    if (rowptr[0] != 0) return fail(KPM_EINVAL, "rowptr[0] must be 0");
    std::vector<int32_t> len(static_cast<size_t>(N));
    for (int64_t i = 0; i < N; ++i) {
        const int64_t l = rowptr[i + 1] - rowptr[i];
        if (l < 0) return fail(KPM_EINVAL, "rowptr decreases at row " + std::to_string(i));
        if (l > INT32_MAX / 64) return fail(KPM_ENOMEM, "a row has too many entries");
        len[i] = static_cast<int32_t>(l);
    }
    perm.resize(static_cast<size_t>(N));
    std::iota(perm.begin(), perm.end(), 0);
    if (sigma > 1) {
        for (int64_t w0 = 0; w0 < N; w0 += sigma) {
            const int64_t w1 = std::min<int64_t>(N, w0 + sigma);
            std::stable_sort(perm.begin() + w0, perm.begin() + w1,
                             [&](int32_t x, int32_t y) { return len[x] > len[y]; });
        }
    }
    const int64_t nch = (N + C - 1) / C;
    width.assign(static_cast<size_t>(nch), 0);
    start.assign(static_cast<size_t>(nch) + 1, 0);
    len_sorted.resize(static_cast<size_t>(N));
    for (int64_t p = 0; p < N; ++p) {
        len_sorted[p] = len[perm[p]];
        width[p / C] = std::max(width[p / C], len_sorted[p]);
    }
    for (int64_t c = 0; c < nch; ++c) start[c + 1] = start[c] + static_cast<int64_t>(width[c]) * C;
    return KPM_OK;
}

// kpm_export_csr of SELL storage: each row's entries in the order they were
// imported (padding dropped, explicit zeros of the input kept).
kpm_status export_sell(const kpm_hamiltonian* H, int64_t* rowptr, int32_t* col, double* val) {
    const SellStore& c = H->sell;
    const int64_t N = H->nrows;
    std::vector<int64_t> pos(static_cast<size_t>(N));   // sorted position of each row
    for (int64_t p = 0; p < N; ++p) pos[c.perm_host.empty() ? p : c.perm_host[p]] = p;
    rowptr[0] = 0;
    for (int64_t i = 0; i < N; ++i) rowptr[i + 1] = rowptr[i] + c.len[pos[i]];
    if (!col) return KPM_OK;
    const size_t n = static_cast<size_t>(c.stored);
    std::vector<int32_t> cc(n);
    std::vector<double> v(2 * n);
    KPM_HIP(hipMemcpy(cc.data(), H->col, n * sizeof(int32_t), hipMemcpyDeviceToHost), "copy col");
    if (H->dtype == KPM_C128) {
        KPM_HIP(hipMemcpy(v.data(), H->val, 2 * n * sizeof(double), hipMemcpyDeviceToHost), "copy val");
    } else {
        std::vector<float> f(2 * n);
        KPM_HIP(hipMemcpy(f.data(), H->val, 2 * n * sizeof(float), hipMemcpyDeviceToHost), "copy val");
        for (size_t i = 0; i < 2 * n; ++i) v[i] = f[i];
    }
    for (int64_t i = 0; i < N; ++i) {
        const int64_t p = pos[i];
        const int64_t e0 = c.start_host[p >> c.clog] + (p & (c.C - 1));
        for (int64_t j = 0, k = rowptr[i]; k < rowptr[i + 1]; ++j, ++k) {
            const int64_t e = e0 + j * c.C;
            col[k] = cc[e];
            val[2 * k] = v[2 * e];
            val[2 * k + 1] = v[2 * e + 1];
        }
    }
    return KPM_OK;
}

}  // namespace

void set_error(const std::string& msg) { g_error = msg; }

}  // namespace kpm

using namespace kpm;

extern "C" {

const char* kpm_last_error(void) { return g_error.c_str(); }

const char* kpm_version(void) { return "kpm-mi355x 0.1 (gfx950)"; }

// A built H handed to SELL-C-sigma storage through host CRS, keeping its
// bounds and scaling.
static kpm_status to_sell(const kpm_hamiltonian* H, int C, int sigma, void* stream, kpm_hamiltonian** out) {
    std::vector<int64_t> rowptr(static_cast<size_t>(H->nrows) + 1);
    kpm_status st = kpm_export_csr(H, rowptr.data(), nullptr, nullptr);
    if (st != KPM_OK) return st;
    const size_t nnz = static_cast<size_t>(rowptr.back());
    std::vector<int32_t> col(nnz > 0 ? nnz : 1);
    std::vector<double> val(nnz > 0 ? 2 * nnz : 2);
    if ((st = kpm_export_csr(H, rowptr.data(), col.data(), val.data())) != KPM_OK) return st;
    kpm_csr_desc c{};
    c.N = H->nrows;
    c.rowptr = rowptr.data();
    c.col = col.data();
    c.val = val.data();
    c.dtype = H->dtype;
    c.sell_C = C;
    c.sell_sigma = sigma;
    c.margin = 1.0;
    c.fixed_scale = 1;
    c.a = H->a;
    c.b = H->b;
    if ((st = kpm_import_csr(&c, stream, out)) != KPM_OK) return st;
    (*out)->emin = H->emin;
    (*out)->emax = H->emax;
    return KPM_OK;
}

kpm_status kpm_build_hamiltonian(const kpm_lattice_desc* d, void* stream, kpm_hamiltonian** out) {
    g_error.clear();
    if (!out) return fail(KPM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d) return fail(KPM_EINVAL, "desc is NULL");
    if (!d->potential && (!std::isfinite(d->gamma) || d->gamma < 0.0))
        return fail(KPM_EINVAL, "gamma must be finite and >= 0 when no potential is given");
    for (int j = 0; j < 3; ++j) {
        if (d->L[j] <= 0) return fail(KPM_EINVAL, "lattice side <= 0");
        if (d->periodic[j] && d->L[j] < 3)
            return fail(KPM_ENOTSUP, "periodic sides must be >= 3 (shorter ones alias the two neighbours)");
    }
    if (d->dtype != KPM_C128 && d->dtype != KPM_C64) return fail(KPM_EINVAL, "unknown dtype");
    if (!std::isfinite(d->t)) return fail(KPM_EINVAL, "t is not finite");
    if (d->fixed_scale) {
        if (!(d->a > 0.0) || !std::isfinite(d->a) || !std::isfinite(d->b))
            return fail(KPM_EINVAL, "fixed scale needs a finite a > 0 and a finite b");
    } else if (!(d->margin >= 1.0) || !std::isfinite(d->margin)) {
        return fail(KPM_EINVAL, "margin must be a finite number >= 1");
    }
    if (d->sell_C != 0) {
        if (d->sell_C < 1 || d->sell_C > 64 || (d->sell_C & (d->sell_C - 1)) != 0)
            return fail(KPM_EINVAL, "sell_C must be 0 or a power of two in 1..64");
        if (d->sell_sigma < 0 || (d->sell_sigma > 1 && d->sell_sigma % d->sell_C != 0))
            return fail(KPM_EINVAL, "sell_sigma must be 0, 1 or a multiple of sell_C");
    }
    const int64_t nsite = static_cast<int64_t>(d->L[0]) * d->L[1] * d->L[2];
    if (nsite > (INT32_MAX / 4)) return fail(KPM_ENOMEM, "lattice too large for int32 column indices");
    if (d->potential)
        for (int64_t i = 0; i < nsite; ++i)
            if (!std::isfinite(d->potential[i])) return fail(KPM_EINVAL, "potential has a non-finite value");

    auto* H = new kpm_hamiltonian();
    hipStream_t s = static_cast<hipStream_t>(stream);
    H->dtype = d->dtype;
    H->nrows = 4 * nsite;
    for (int j = 0; j < 3; ++j) {
        H->L[j] = d->L[j];
        H->periodic[j] = d->periodic[j] ? 1 : 0;
    }
    H->width = kWidth;
    if (hipGetDevice(&H->device) != hipSuccess) {
        delete H;
        return fail(KPM_EDEVICE, "hipGetDevice failed");
    }
    const size_t slots = static_cast<size_t>(H->nrows) * kWidth;
    const int nblocks = build_blocks(H->nrows);
    double* pot_dev = nullptr;
    double* bb = nullptr;
    double* bounds = nullptr;
    double host_bounds[2] = {0.0, 0.0};
    kpm_status st = KPM_OK;
    hipError_t e;
    if ((e = hipMalloc(&H->val, slots * 2 * real_size(H->dtype))) != hipSuccess) st = hip_fail(e, "hipMalloc(val)");
    else if ((e = hipMalloc(&H->col, slots * sizeof(int32_t))) != hipSuccess) st = hip_fail(e, "hipMalloc(col)");
    else if ((e = hipMalloc(&pot_dev, nsite * sizeof(double))) != hipSuccess) st = hip_fail(e, "hipMalloc(potential)");
    else if ((e = hipMalloc(&bb, static_cast<size_t>(nblocks) * 2 * sizeof(double))) != hipSuccess) st = hip_fail(e, "hipMalloc(bounds)");
    else if ((e = hipMalloc(&bounds, 2 * sizeof(double))) != hipSuccess) st = hip_fail(e, "hipMalloc(bounds)");
    else if (d->potential &&
             (e = hipMemcpyAsync(pot_dev, d->potential, nsite * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess)
        st = hip_fail(e, "copy potential");
    else if (!d->potential && (e = launch_potential(pot_dev, nsite, d->gamma, d->seed, s)) != hipSuccess)
        st = hip_fail(e, "potential kernel");
    else if ((e = launch_build_ti(d->L[0], d->L[1], d->L[2], d->periodic, d->t, pot_dev, H->dtype, H->val,
                                  H->col, bb, nblocks, bounds, s)) != hipSuccess)
        st = hip_fail(e, "build kernel");
    else if ((e = hipMemcpyAsync(host_bounds, bounds, 2 * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess)
        st = hip_fail(e, "copy bounds");
    else if ((e = hipStreamSynchronize(s)) != hipSuccess)
        st = hip_fail(e, "synchronise");
    if (pot_dev) (void)hipFree(pot_dev);
    if (bb) (void)hipFree(bb);
    if (bounds) (void)hipFree(bounds);
    if (st != KPM_OK) {
        kpm_destroy_hamiltonian(H);
        return st;
    }
    H->emin = host_bounds[0];
    H->emax = host_bounds[1];
    if (d->fixed_scale) {
        H->a = d->a;
        H->b = d->b;
    } else {
        H->b = 0.5 * (H->emax + H->emin);
        H->a = d->margin * 0.5 * (H->emax - H->emin);
        if (!(H->a > 0.0)) {
            kpm_destroy_hamiltonian(H);
            return fail(KPM_EINVAL, "Gershgorin interval has zero width");
        }
    }
    if (d->sell_C > 0) {
        // the built matrix into SELL-C-sigma storage, with the lattice's
        // bounds and scaling (those of the exact entries)
        kpm_hamiltonian* S = nullptr;
        st = to_sell(H, d->sell_C, d->sell_sigma, stream, &S);
        kpm_destroy_hamiltonian(H);
        if (st != KPM_OK) return st;
        H = S;
    }
    *out = H;
    return KPM_OK;
}

kpm_status kpm_hamiltonian_info(const kpm_hamiltonian* H, int64_t* N, int64_t* nnz, int32_t* width,
                                int32_t* dtype, double* a, double* b, double* emin, double* emax) {
    g_error.clear();
    if (!H) return fail(KPM_EINVAL, "H is NULL");
    if (N) *N = H->nrows;
    if (nnz) *nnz = H->sell.C > 0 ? H->sell.stored : H->nrows * H->width;
    if (width) *width = H->width;
    if (dtype) *dtype = H->dtype;
    if (a) *a = H->a;
    if (b) *b = H->b;
    if (emin) *emin = H->emin;
    if (emax) *emax = H->emax;
    return KPM_OK;
}

kpm_status kpm_export_csr(const kpm_hamiltonian* H, int64_t* rowptr, int32_t* col, double* val) {
    g_error.clear();
    if (!H || !rowptr) return fail(KPM_EINVAL, "H or rowptr is NULL");
    if ((col == nullptr) != (val == nullptr)) return fail(KPM_EINVAL, "col and val must both be set or both NULL");
    kpm_status st = check_device(H);
    if (st != KPM_OK) return st;
    if (H->sell.C > 0) return export_sell(H, rowptr, col, val);
    const size_t slots = static_cast<size_t>(H->nrows) * H->width;
    std::vector<int32_t> c(slots);
    std::vector<double> v(2 * slots);
    KPM_HIP(hipMemcpy(c.data(), H->col, slots * sizeof(int32_t), hipMemcpyDeviceToHost), "copy col");
    if (H->dtype == KPM_C128) {
        KPM_HIP(hipMemcpy(v.data(), H->val, 2 * slots * sizeof(double), hipMemcpyDeviceToHost), "copy val");
    } else {
        std::vector<float> f(2 * slots);
        KPM_HIP(hipMemcpy(f.data(), H->val, 2 * slots * sizeof(float), hipMemcpyDeviceToHost), "copy val");
        for (size_t i = 0; i < 2 * slots; ++i) v[i] = f[i];
    }
    int64_t k = 0;
    rowptr[0] = 0;
    for (int64_t i = 0; i < H->nrows; ++i) {
        for (int j = 0; j < H->width; ++j) {
            const size_t s = static_cast<size_t>(i) * H->width + j;
            if (j > 0 && c[s] == i) continue;   // padding slot
            if (col) {
                col[k] = c[s];
                val[2 * k] = v[2 * s];
                val[2 * k + 1] = v[2 * s + 1];
            }
            ++k;
        }
        rowptr[i + 1] = k;
    }
    return KPM_OK;
}

void kpm_destroy_hamiltonian(kpm_hamiltonian* H) {
    if (!H) return;
    (void)hipDeviceSynchronize();
    if (H->val) (void)hipFree(H->val);
    if (H->col) (void)hipFree(H->col);
    if (H->sell.start) (void)hipFree(H->sell.start);
    if (H->sell.width) (void)hipFree(H->sell.width);
    if (H->sell.perm) (void)hipFree(H->sell.perm);
    for (auto& kv : H->ws) free_workspace(kv.second);
    for (auto& kv : H->sched) (void)hipFree(kv.second);
    delete H;
}

kpm_status kpm_sell_layout(int64_t N, const int64_t* rowptr, int32_t C, int32_t sigma, int32_t* perm,
                           int32_t* width, int64_t* start) {
    g_error.clear();
    std::vector<int32_t> pm, wd, ln;
    std::vector<int64_t> st;
    const kpm_status e = sell_layout(N, rowptr, C, sigma, pm, wd, st, ln);
    if (e != KPM_OK) return e;
    if (perm) std::copy(pm.begin(), pm.end(), perm);
    if (width) std::copy(wd.begin(), wd.end(), width);
    if (start) std::copy(st.begin(), st.end(), start);
    return KPM_OK;
}

kpm_status kpm_import_csr(const kpm_csr_desc* d, void* stream, kpm_hamiltonian** out) {
    g_error.clear();
    if (!out) return fail(KPM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d) return fail(KPM_EINVAL, "desc is NULL");
    if (d->dtype != KPM_C128 && d->dtype != KPM_C64) return fail(KPM_EINVAL, "unknown dtype");
    if (d->fixed_scale) {
        if (!(d->a > 0.0) || !std::isfinite(d->a) || !std::isfinite(d->b))
            return fail(KPM_EINVAL, "fixed scale needs a finite a > 0 and a finite b");
    } else if (!(d->margin >= 1.0) || !std::isfinite(d->margin)) {
        return fail(KPM_EINVAL, "margin must be a finite number >= 1");
    }
    const int C = d->sell_C == 0 ? 8 : d->sell_C;
    const int sigma = d->sell_sigma == 0 ? 128 * C : d->sell_sigma;
    std::vector<int32_t> perm, width, len;
    std::vector<int64_t> start;
    kpm_status st = sell_layout(d->N, d->rowptr, C, sigma, perm, width, start, len);
    if (st != KPM_OK) return st;
    const int64_t N = d->N;
    const int64_t nnz = d->rowptr[N];
    if (nnz > 0 && (!d->col || !d->val)) return fail(KPM_EINVAL, "col or val is NULL");
    for (int64_t k = 0; k < nnz; ++k)
        if (d->col[k] < 0 || d->col[k] >= N) return fail(KPM_EINVAL, "column out of range at entry " + std::to_string(k));
    for (int64_t k = 0; k < 2 * nnz; ++k)
        if (!std::isfinite(d->val[k])) return fail(KPM_EINVAL, "non-finite value at entry " + std::to_string(k / 2));
    const int64_t nch = static_cast<int64_t>(width.size());
    const int64_t stored = start[nch];
    const size_t rs = real_size(d->dtype);
    if (static_cast<uint64_t>(stored) * 2 * rs >= (1ull << 32) - 64)
        return fail(KPM_ENOMEM, "SELL storage reaches 4 GiB of values");

    // the padded arrays: value 0 and column N wherever a row ends early
    const size_t ns = static_cast<size_t>(stored > 0 ? stored : 1);
    std::vector<int32_t> hcol(ns, static_cast<int32_t>(N));
    std::vector<double> hval(d->dtype == KPM_C128 ? 2 * ns : 0, 0.0);
    std::vector<float> fval(d->dtype == KPM_C64 ? 2 * ns : 0, 0.0f);
    for (int64_t p = 0; p < N; ++p) {
        const int64_t row = perm[p];
        const int64_t e0 = start[p / C] + (p % C);
        for (int64_t k = d->rowptr[row], j = 0; k < d->rowptr[row + 1]; ++k, ++j) {
            const int64_t e = e0 + j * C;
            hcol[e] = d->col[k];
            if (d->dtype == KPM_C128) {
                hval[2 * e] = d->val[2 * k];
                hval[2 * e + 1] = d->val[2 * k + 1];
            } else {
                fval[2 * e] = static_cast<float>(d->val[2 * k]);
                fval[2 * e + 1] = static_cast<float>(d->val[2 * k + 1]);
            }
        }
    }

    auto* H = new kpm_hamiltonian();
    hipStream_t s = static_cast<hipStream_t>(stream);
    H->dtype = d->dtype;
    H->nrows = N;
    H->width = nch > 0 ? *std::max_element(width.begin(), width.end()) : 0;
    SellStore& c = H->sell;
    c.C = C;
    c.clog = 0;
    while ((1 << c.clog) < C) ++c.clog;
    c.sigma = sigma;
    c.nchunks = nch;
    c.stored = stored;
    c.nnz = nnz;
    c.len = std::move(len);
    c.start_host = start;
    if (sigma > 1) c.perm_host = perm;
    if (hipGetDevice(&H->device) != hipSuccess) {
        delete H;
        return fail(KPM_EDEVICE, "hipGetDevice failed");
    }
    const int nblocks = build_blocks(N);
    double* bb = nullptr;
    double* bounds = nullptr;
    double host_bounds[2] = {0.0, 0.0};
    hipError_t e;
    const size_t vbytes = ns * 2 * rs;
    if ((e = hipMalloc(&H->val, vbytes)) != hipSuccess) st = hip_fail(e, "hipMalloc(val)");
    else if ((e = hipMalloc(&H->col, ns * sizeof(int32_t))) != hipSuccess) st = hip_fail(e, "hipMalloc(col)");
    else if ((e = hipMalloc(&c.start, start.size() * sizeof(int64_t))) != hipSuccess) st = hip_fail(e, "hipMalloc(start)");
    else if ((e = hipMalloc(&c.width, width.size() * sizeof(int32_t))) != hipSuccess) st = hip_fail(e, "hipMalloc(width)");
    else if (sigma > 1 && (e = hipMalloc(&c.perm, perm.size() * sizeof(int32_t))) != hipSuccess)
        st = hip_fail(e, "hipMalloc(perm)");
    else if ((e = hipMalloc(&bb, static_cast<size_t>(nblocks) * 2 * sizeof(double))) != hipSuccess)
        st = hip_fail(e, "hipMalloc(bounds)");
    else if ((e = hipMalloc(&bounds, 2 * sizeof(double))) != hipSuccess) st = hip_fail(e, "hipMalloc(bounds)");
    else if ((e = hipMemcpyAsync(H->val, d->dtype == KPM_C128 ? static_cast<const void*>(hval.data()) : fval.data(),
                                 vbytes, hipMemcpyHostToDevice, s)) != hipSuccess)
        st = hip_fail(e, "copy val");
    else if ((e = hipMemcpyAsync(H->col, hcol.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice, s)) != hipSuccess)
        st = hip_fail(e, "copy col");
    else if ((e = hipMemcpyAsync(c.start, start.data(), start.size() * sizeof(int64_t), hipMemcpyHostToDevice, s)) !=
             hipSuccess)
        st = hip_fail(e, "copy start");
    else if ((e = hipMemcpyAsync(c.width, width.data(), width.size() * sizeof(int32_t), hipMemcpyHostToDevice, s)) !=
             hipSuccess)
        st = hip_fail(e, "copy width");
    else if (sigma > 1 && (e = hipMemcpyAsync(c.perm, perm.data(), perm.size() * sizeof(int32_t),
                                              hipMemcpyHostToDevice, s)) != hipSuccess)
        st = hip_fail(e, "copy perm");
    else if ((e = launch_sell_bounds(H->dtype, H->val, H->col, c.start, c.width, c.perm, N, c.clog, bb, bounds, s)) !=
             hipSuccess)
        st = hip_fail(e, "bounds kernel");
    else if ((e = hipMemcpyAsync(host_bounds, bounds, 2 * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess)
        st = hip_fail(e, "copy bounds");
    else if ((e = hipStreamSynchronize(s)) != hipSuccess)
        st = hip_fail(e, "synchronise");
    if (bb) (void)hipFree(bb);
    if (bounds) (void)hipFree(bounds);
    if (st != KPM_OK) {
        kpm_destroy_hamiltonian(H);
        return st;
    }
    H->emin = host_bounds[0];
    H->emax = host_bounds[1];
    if (d->fixed_scale) {
        H->a = d->a;
        H->b = d->b;
    } else {
        H->b = 0.5 * (H->emax + H->emin);
        H->a = d->margin * 0.5 * (H->emax - H->emin);
        if (!(H->a > 0.0)) {
            kpm_destroy_hamiltonian(H);
            return fail(KPM_EINVAL, "Gershgorin interval has zero width");
        }
    }
    *out = H;
    return KPM_OK;
}

kpm_status kpm_sell_info(const kpm_hamiltonian* H, int32_t* C, int32_t* sigma, int64_t* nchunks, int64_t* stored,
                         int64_t* nnz) {
    g_error.clear();
    if (!H) return fail(KPM_EINVAL, "H is NULL");
    const SellStore& c = H->sell;
    if (C) *C = c.C;
    if (sigma) *sigma = c.C > 0 ? c.sigma : 0;
    if (nchunks) *nchunks = c.nchunks;
    if (stored) *stored = c.stored;
    if (nnz) *nnz = c.nnz;
    return KPM_OK;
}

kpm_status kpm_aug_spmmv(const kpm_hamiltonian* Hc, const void* V, void* W, int32_t R, double alpha,
                         double beta, double gamma, int32_t variant, double* eta, void* stream) {
    g_error.clear();
    if (!Hc || !V || !W) return fail(KPM_EINVAL, "H, V or W is NULL");
    if (!r_supported(R)) return fail(KPM_ENOTSUP, "R must be one of 1, 2, 4, 8, 16, 32, 64");
    if (variant != KPM_FULL && variant != KPM_NODOT && variant != KPM_PLAIN)
        return fail(KPM_EINVAL, "unknown variant");
    if (!std::isfinite(alpha) || !std::isfinite(beta) || !std::isfinite(gamma))
        return fail(KPM_EINVAL, "alpha, beta, gamma must be finite");
    auto* H = const_cast<kpm_hamiltonian*>(Hc);
    kpm_status st = check_device(H);
    if (st != KPM_OK) return st;
    if ((st = check_sell_block(H, R)) != KPM_OK) return st;
    const size_t bytes = static_cast<size_t>(H->nrows) * 2 * R * real_size(H->dtype);
    const char* v0 = static_cast<const char*>(V);
    const char* w0 = static_cast<const char*>(W);
    if (v0 < w0 + bytes && w0 < v0 + bytes) return fail(KPM_EINVAL, "V and W overlap");
    TuningScope scope(nullptr);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace& w = *workspace(H, s);
    const int32_t* sched = nullptr;
    if ((st = schedule_for(H, &sched)) != KPM_OK) return st;
    const bool dots = (variant == KPM_FULL && eta != nullptr);
    if (dots) {
        st = ensure_partials(w, H, R, 1);
        if (st != KPM_OK) return st;
    }
    if ((st = ensure_queue(w)) != KPM_OK) return st;
    if (sweep_uses_queue(H, R)) KPM_HIP(launch_zero_ints(w.queue, kXcds, s), "zero kernel");
    SweepArgs a{H->val, H->col, H->nrows, V, W, sched, alpha, beta, gamma,
                dots ? w.partials : nullptr, launch_grid(H, R)};
    a.queue = w.queue;
    for (int j = 0; j < 3; ++j) a.L[j] = H->L[j];
    const int launch_variant = (variant == KPM_FULL && !dots) ? KPM_NODOT : variant;
    KPM_HIP(launch_any_sweep(H, R, launch_variant, a, s), "sweep kernel");
    if (dots) KPM_HIP(launch_reduce_partials(w.partials, 1, a.grid, R, 0, eta, s), "reduce kernel");
    return KPM_OK;
}

kpm_status kpm_moments(const kpm_hamiltonian* Hc, const void* V0, int32_t R, int32_t M, double* mu,
                       const kpm_run_opts* opts_in, void* stream) {
    g_error.clear();
    const kpm_run_opts opts = opts_in ? *opts_in : kpm_run_opts{};
    if (!Hc || !V0) return fail(KPM_EINVAL, "H or V0 is NULL");
    if (opts.variant != KPM_FULL && opts.variant != KPM_NODOT)
        return fail(KPM_EINVAL, "kpm_moments runs the FULL or the NODOT variant");
    const bool full = opts.variant == KPM_FULL;
    if (full && !mu) return fail(KPM_EINVAL, "mu is NULL");
    if (!r_supported(R)) return fail(KPM_ENOTSUP, "R must be one of 1, 2, 4, 8, 16, 32, 64");
    if (M < 2 || (M % 2) != 0) return fail(KPM_EINVAL, "M must be even and >= 2");
    if (reinterpret_cast<uintptr_t>(V0) % 16 != 0) return fail(KPM_EINVAL, "V0 must be 16-byte aligned");
    kpm_status st;
    if (opts.tuning && (st = check_tuning(*opts.tuning)) != KPM_OK) return st;
    auto* H = const_cast<kpm_hamiltonian*>(Hc);
    if ((st = check_device(H)) != KPM_OK) return st;
    // column groups: the caller's width, or the widest supported width whose
    // block the sweeps can address (32-bit buffer offsets, the padding row
    // of imported matrices included)
    int G = default_group(H, R, opts.eta_out == nullptr);
    if (opts.group != 0) {
        if (!r_supported(opts.group) || R % opts.group != 0)
            return fail(KPM_EINVAL, "group must be one of 1, 2, 4, ..., 64 and divide R");
        G = opts.group;
    }
    const bool grouped = G < R;
    if (grouped && opts.eta_out) return fail(KPM_ENOTSUP, "eta_out needs the whole block in one recurrence");
    if ((st = check_sell_block(H, G)) != KPM_OK) return st;
    TuningScope scope(opts.tuning);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace& w = *workspace(H, s);
    const int sweeps = M / 2;
    const int slots = sweeps < kReduceEvery ? sweeps : kReduceEvery;
    const int32_t* sched = nullptr;
    if ((st = ensure_vectors(w, H, G)) != KPM_OK) return st;
    if ((st = schedule_for(H, &sched)) != KPM_OK) return st;
    if (full && (st = ensure_partials(w, H, G, slots)) != KPM_OK) return st;
    if ((st = ensure_queue(w)) != KPM_OK) return st;
    double* eta = opts.eta_out;
    if (full && !eta) {
        if ((st = grow(&w.eta, &w.etabytes, static_cast<size_t>(M) * G * 2 * sizeof(double), "hipMalloc(eta)")) !=
            KPM_OK)
            return st;
        eta = w.eta;
    }
    double* mu_dev = mu;
    if (full && opts.mu_on_host) {
        if ((st = grow(&w.mu, &w.mubytes, static_cast<size_t>(M) * R * sizeof(double), "hipMalloc(mu)")) != KPM_OK)
            return st;
        mu_dev = w.mu;
    }
    if (full && opts.check && (st = ensure_flag(w)) != KPM_OK) return st;
    const int grid = launch_grid(H, G);
    const size_t slot_elems = static_cast<size_t>(grid) * 3 * G;
    const size_t bytes = static_cast<size_t>(H->nrows) * 2 * R * real_size(H->dtype);
    void* A = w.vbuf[0];
    void* B = w.vbuf[1];
    const double inv_a = 1.0 / H->a, b = H->b;
    const int variant = opts.variant;

    // the launch sequence of one call, on stream q: per column group, its
    // start vectors into A, the M/2 sweeps, the reductions and eta -> mu
    auto enqueue = [&](hipStream_t q, bool capturing) -> kpm_status {
        for (int c0 = 0; c0 < R; c0 += G) {
            // nu_0 -> A (the caller's block stays untouched)
            if (grouped) KPM_HIP(launch_columns(H->dtype, H->nrows, R, c0, G, V0, A, q), "copy V0 columns");
            else KPM_HIP(launch_copy16(A, V0, bytes, q), "copy V0");
            for (int k = 0; k < sweeps; ++k) {
                const int sl = k % kReduceEvery;
                if (sl == 0)   // tile counters of the next kReduceEvery sweeps
                    KPM_HIP(launch_zero_ints(w.queue, kReduceEvery * kXcds, q), "zero kernel");
                SweepArgs a{H->val, H->col, H->nrows, nullptr, nullptr, sched, 0.0, 0.0, 0.0,
                            full ? w.partials + sl * slot_elems : nullptr, grid};
                a.queue = w.queue + sl * kXcds;
                for (int j = 0; j < 3; ++j) a.L[j] = H->L[j];
                if (k == 0) {
                    // nu_1 = Htilde nu_0 = (1/a) H nu_0 - (b/a) nu_0
                    a.V = A; a.W = B; a.alpha = inv_a; a.beta = -b * inv_a; a.gamma = 0.0;
                } else {
                    // swap roles: V = nu_k, W = nu_{k-1} -> nu_{k+1} = 2 Htilde nu_k - nu_{k-1}
                    if (k % 2 == 1) { a.V = B; a.W = A; } else { a.V = A; a.W = B; }
                    a.alpha = 2.0 * inv_a; a.beta = -2.0 * b * inv_a; a.gamma = -1.0;
                }
                KPM_HIP(launch_any_sweep(H, G, variant, a, q, capturing), "sweep kernel");
                if (full && (sl == kReduceEvery - 1 || k == sweeps - 1))
                    KPM_HIP(launch_reduce_partials(w.partials, sl + 1, grid, G, k - sl, eta, q), "reduce kernel");
            }
            if (full)
                KPM_HIP(launch_eta_to_mu(eta, G, M, mu_dev + static_cast<size_t>(c0) * M, q), "eta_to_mu kernel");
        }
        return KPM_OK;
    };

    if (opts.use_graph) {
        std::vector<unsigned char> key;
        const kpm_sweep_tuning t = get_tuning();
        key_add(key, V0); key_add(key, mu_dev); key_add(key, eta); key_add(key, R); key_add(key, G); key_add(key, M);
        key_add(key, H->a); key_add(key, H->b); key_add(key, variant); key_add(key, t); key_add(key, grid);
        key_add(key, A); key_add(key, B); key_add(key, w.partials); key_add(key, w.queue); key_add(key, sched);
        if (!w.exec || w.graph_key != key) {
            drop_moments_graph(w);
            if (!w.capture) KPM_HIP(hipStreamCreateWithFlags(&w.capture, hipStreamNonBlocking), "hipStreamCreate");
            KPM_HIP(hipStreamBeginCapture(w.capture, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            const kpm_status se = enqueue(w.capture, true);
            hipGraph_t g = nullptr;
            const hipError_t ee = hipStreamEndCapture(w.capture, &g);
            if (se != KPM_OK) {
                if (g) (void)hipGraphDestroy(g);
                return se;
            }
            if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
            w.graph = g;
            const hipError_t ei = hipGraphInstantiate(&w.exec, w.graph, nullptr, nullptr, 0);
            if (ei != hipSuccess) {
                drop_moments_graph(w);
                return hip_fail(ei, "hipGraphInstantiate");
            }
            w.graph_key = key;
        }
        KPM_HIP(hipGraphLaunch(w.exec, s), "hipGraphLaunch");
    } else if ((st = enqueue(s, false)) != KPM_OK) {
        return st;
    }
    if (full && opts.check) {
        KPM_HIP(launch_check_moments(mu_dev, R, M, w.flag, s), "check kernel");
        KPM_HIP(hipMemcpyAsync(w.flag_host, w.flag, sizeof(int), hipMemcpyDeviceToHost, s), "copy flag");
        KPM_HIP(hipStreamSynchronize(s), "synchronise");
        if (*w.flag_host)
            return fail(KPM_ESPECTRUM, "moments left [-mu_0, mu_0]: the scaled spectrum is not inside [-1, 1]");
    }
    if (full && opts.mu_on_host) {
        KPM_HIP(hipMemcpyAsync(mu, mu_dev, static_cast<size_t>(M) * R * sizeof(double), hipMemcpyDeviceToHost, s),
                "copy mu");
        KPM_HIP(hipStreamSynchronize(s), "synchronise");
    }
    return KPM_OK;
}

kpm_status kpm_moments_naive(const kpm_hamiltonian* Hc, const void* V0, int32_t R, int32_t M, double* mu,
                             int32_t check, void* stream) {
    g_error.clear();
    if (!Hc || !V0 || !mu) return fail(KPM_EINVAL, "H, V0 or mu is NULL");
    if (!r_supported(R)) return fail(KPM_ENOTSUP, "R must be one of 1, 2, 4, 8, 16, 32, 64");
    if (M < 2 || (M % 2) != 0) return fail(KPM_EINVAL, "M must be even and >= 2");
    auto* H = const_cast<kpm_hamiltonian*>(Hc);
    kpm_status st = check_device(H);
    if (st != KPM_OK) return st;
    if ((st = check_sell_block(H, 1)) != KPM_OK) return st;
    TuningScope scope(nullptr);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace& ws = *workspace(H, s);
    const int32_t* sched = nullptr;
    if ((st = schedule_for(H, &sched)) != KPM_OK) return st;
    const int64_t N = H->nrows;
    const size_t vb = static_cast<size_t>(N) * 2 * real_size(H->dtype);
    for (int i = 0; i < 3; ++i) {
        size_t have = ws.naive_bytes;
        if ((st = grow(&ws.naive[i], &have, vb, "hipMalloc(naive vector)")) != KPM_OK) return st;
    }
    ws.naive_bytes = vb;
    if (!ws.dot_part)
        KPM_HIP(hipMalloc(&ws.dot_part, static_cast<size_t>(naive_dot_partials()) * 2 * sizeof(double)),
                "hipMalloc(dot partials)");
    if ((st = grow(&ws.eta, &ws.etabytes, static_cast<size_t>(M) * R * 2 * sizeof(double), "hipMalloc(eta)")) !=
        KPM_OK)
        return st;
    double* eta = ws.eta;   // [M][R][2]
    const int dt = H->dtype;
    const double inv_a = 1.0 / H->a, b = H->b;
    // one SpMV: u <- H v (the plain sweep at R = 1, which applies H unscaled)
    auto spmv = [&](const void* v, void* u) -> hipError_t {
        SweepArgs a{H->val, H->col, N, v, u, sched, 1.0, 0.0, 0.0, nullptr, launch_grid(H, 1)};
        a.queue = ws.queue;
        for (int j = 0; j < 3; ++j) a.L[j] = H->L[j];
        if (sweep_uses_queue(H, 1)) {
            const hipError_t e = launch_zero_ints(ws.queue, kXcds, s);
            if (e != hipSuccess) return e;
        }
        return launch_any_sweep(H, 1, KPM_PLAIN, a, s);
    };
    auto eta_at = [&](int n, int r) { return eta + (static_cast<int64_t>(n) * R + r) * 2; };
    if ((st = ensure_queue(ws)) != KPM_OK) return st;
    // the stochastic trace as an outer loop over the R start vectors
    for (int r = 0; r < R; ++r) {
        void* v = ws.naive[0];
        void* w = ws.naive[1];
        void* u = ws.naive[2];
        KPM_HIP(launch_column(dt, N, R, r, V0, v, s), "column kernel");
        // initialisation: w = nu_1 = (H v - b v) / a; eta_0 = <v|v>, eta_1 = <w|v>
        KPM_HIP(spmv(v, w), "spmv");
        KPM_HIP(launch_axpy(dt, N, -b, v, w, s), "axpy kernel");
        KPM_HIP(launch_scal(dt, N, inv_a, w, s), "scal kernel");
        KPM_HIP(launch_dot(dt, N, v, v, ws.dot_part, eta_at(0, r), s), "nrm2 kernel");
        KPM_HIP(launch_dot(dt, N, w, v, ws.dot_part, eta_at(1, r), s), "dot kernel");
        for (int m = 1; m < M / 2; ++m) {
            std::swap(v, w);   // v = nu_m, w = nu_{m-1}
            KPM_HIP(spmv(v, u), "spmv");
            KPM_HIP(launch_axpy(dt, N, -b, v, u, s), "axpy kernel");
            KPM_HIP(launch_scal(dt, N, -1.0, w, s), "scal kernel");
            KPM_HIP(launch_axpy(dt, N, 2.0 * inv_a, u, w, s), "axpy kernel");
            KPM_HIP(launch_dot(dt, N, v, v, ws.dot_part, eta_at(2 * m, r), s), "nrm2 kernel");
            KPM_HIP(launch_dot(dt, N, w, v, ws.dot_part, eta_at(2 * m + 1, r), s), "dot kernel");
        }
    }
    KPM_HIP(launch_eta_to_mu(eta, R, M, mu, s), "eta_to_mu kernel");
    if (check) {
        if ((st = ensure_flag(ws)) != KPM_OK) return st;
        KPM_HIP(launch_check_moments(mu, R, M, ws.flag, s), "check kernel");
        KPM_HIP(hipMemcpyAsync(ws.flag_host, ws.flag, sizeof(int), hipMemcpyDeviceToHost, s), "copy flag");
        KPM_HIP(hipStreamSynchronize(s), "synchronise");
        if (*ws.flag_host)
            return fail(KPM_ESPECTRUM, "moments left [-mu_0, mu_0]: the scaled spectrum is not inside [-1, 1]");
    }
    return KPM_OK;
}

kpm_status kpm_lanczos_bounds(const kpm_hamiltonian* Hc, int32_t steps, uint64_t seed, double* emin, double* emax,
                              void* stream) {
    g_error.clear();
    if (!Hc || !emin || !emax) return fail(KPM_EINVAL, "H, emin or emax is NULL");
    if (steps < 2 || steps > lanczos_max_steps()) return fail(KPM_EINVAL, "steps must be in [2, 1024]");
    auto* H = const_cast<kpm_hamiltonian*>(Hc);
    kpm_status st = check_device(H);
    if (st != KPM_OK) return st;
    if ((st = check_sell_block(H, 1)) != KPM_OK) return st;
    TuningScope scope(nullptr);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace& ws = *workspace(H, s);
    const int32_t* sched = nullptr;
    if ((st = schedule_for(H, &sched)) != KPM_OK) return st;
    const int64_t N = H->nrows;
    const int dt = H->dtype;
    const size_t vb = static_cast<size_t>(N) * 2 * real_size(dt);
    for (int i = 0; i < 3; ++i) {
        size_t have = ws.naive_bytes;
        if ((st = grow(&ws.naive[i], &have, vb, "hipMalloc(Lanczos vector)")) != KPM_OK) return st;
    }
    ws.naive_bytes = vb;
    if (!ws.dot_part)
        KPM_HIP(hipMalloc(&ws.dot_part, static_cast<size_t>(naive_dot_partials()) * 2 * sizeof(double)),
                "hipMalloc(dot partials)");
    // [steps][2] (alpha_j, beta_{j-1}), [steps] beta_j, <q|Hq>, |w|^2, the two extremes
    const size_t nd = 3 * static_cast<size_t>(steps) + 6;
    if ((st = grow(&ws.lanczos, &ws.lanczos_bytes, nd * sizeof(double), "hipMalloc(Lanczos scalars)")) != KPM_OK)
        return st;
    if ((st = ensure_queue(ws)) != KPM_OK) return st;
    double* ab = ws.lanczos;
    double* beta = ab + 2 * steps;
    double* dq = beta + steps;
    double* nrm = dq + 2;
    double* ext = nrm + 2;
    void* qp = ws.naive[0];
    void* q = ws.naive[1];
    void* w = ws.naive[2];
    // q_0 = 0 (its coefficient is 0 in the first step, but 0 * garbage need not be 0)
    const int64_t words = static_cast<int64_t>(vb / sizeof(int));
    if (words > INT32_MAX) return fail(KPM_ENOTSUP, "Lanczos vector too large");
    KPM_HIP(launch_zero_ints(static_cast<int*>(qp), static_cast<int>(words), s), "zero kernel");
    // q_1: a random-phase unit vector
    KPM_HIP(launch_phase_block(q, N, 1, dt, seed, s), "phase block kernel");
    for (int j = 0; j < steps; ++j) {
        SweepArgs a{H->val, H->col, N, q, w, sched, 1.0, 0.0, 0.0, nullptr, launch_grid(H, 1)};
        a.queue = ws.queue;
        for (int i = 0; i < 3; ++i) a.L[i] = H->L[i];
        if (sweep_uses_queue(H, 1)) KPM_HIP(launch_zero_ints(ws.queue, kXcds, s), "zero kernel");
        KPM_HIP(launch_any_sweep(H, 1, KPM_PLAIN, a, s), "spmv");                       // w = H q
        KPM_HIP(launch_dot(dt, N, q, w, ws.dot_part, dq, s), "dot kernel");           // alpha_j
        KPM_HIP(launch_lanczos_update(dt, N, dq, j > 0 ? beta + j - 1 : nullptr, ab + 2 * j, q, qp, w, s),
                "update kernel");                                                         // w -= alpha q + beta qp
        KPM_HIP(launch_dot(dt, N, w, w, ws.dot_part, nrm, s), "nrm2 kernel");         // beta_j^2
        KPM_HIP(launch_lanczos_normalise(dt, N, nrm, w, qp, beta + j, s), "normalise kernel");
        std::swap(qp, q);   // q_{j-1} <- q_j, q_j <- q_{j+1}
    }
    KPM_HIP(launch_tridiag_extremes(ab, beta, steps, ext, s), "tridiagonal kernel");
    double host[2];
    KPM_HIP(hipMemcpyAsync(host, ext, sizeof(host), hipMemcpyDeviceToHost, s), "copy extremes");
    KPM_HIP(hipStreamSynchronize(s), "synchronise");
    *emin = host[0];
    *emax = host[1];
    return KPM_OK;
}

kpm_status kpm_set_scaling(kpm_hamiltonian* H, double a, double b) {
    g_error.clear();
    if (!H) return fail(KPM_EINVAL, "H is NULL");
    if (!(a > 0.0) || !std::isfinite(a) || !std::isfinite(b)) return fail(KPM_EINVAL, "need finite a > 0 and finite b");
    H->a = a;
    H->b = b;
    return KPM_OK;
}

namespace {
// scalar-product partials of kpm_dot, one buffer per (device, stream), kept
// until the process ends
std::mutex g_dot_lock;
std::map<std::pair<int, hipStream_t>, double*> g_dot_part;

kpm_status blas1_args(int32_t dtype, int64_t n, std::initializer_list<const void*> ptrs) {
    if (dtype != KPM_C128 && dtype != KPM_C64) return fail(KPM_EINVAL, "unknown dtype");
    if (n < 0) return fail(KPM_EINVAL, "n must be >= 0");
    for (const void* p : ptrs) {
        if (!p && n > 0) return fail(KPM_EINVAL, "NULL vector");
        if (reinterpret_cast<uintptr_t>(p) % 16 != 0) return fail(KPM_EINVAL, "vectors must be 16-byte aligned");
    }
    return KPM_OK;
}
}  // namespace

kpm_status kpm_axpy(int32_t dtype, int64_t n, double alpha, const void* x, void* y, void* stream) {
    g_error.clear();
    kpm_status st = blas1_args(dtype, n, {x, y});
    if (st != KPM_OK || n == 0) return st;
    KPM_HIP(launch_axpy(dtype, n, alpha, x, y, static_cast<hipStream_t>(stream)), "axpy kernel");
    return KPM_OK;
}

kpm_status kpm_scal(int32_t dtype, int64_t n, double alpha, void* x, void* stream) {
    g_error.clear();
    kpm_status st = blas1_args(dtype, n, {x});
    if (st != KPM_OK || n == 0) return st;
    KPM_HIP(launch_scal(dtype, n, alpha, x, static_cast<hipStream_t>(stream)), "scal kernel");
    return KPM_OK;
}

kpm_status kpm_dot(int32_t dtype, int64_t n, const void* x, const void* y, double* out, void* stream) {
    g_error.clear();
    kpm_status st = blas1_args(dtype, n, {x, y});
    if (st != KPM_OK) return st;
    if (!out) return fail(KPM_EINVAL, "out is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    KPM_HIP(hipGetDevice(&dev), "hipGetDevice");
    double* part = nullptr;
    {
        std::lock_guard<std::mutex> g(g_dot_lock);
        double*& p = g_dot_part[{dev, s}];
        if (!p)
            KPM_HIP(hipMalloc(&p, static_cast<size_t>(naive_dot_partials()) * 2 * sizeof(double)),
                    "hipMalloc(dot partials)");
        part = p;
    }
    KPM_HIP(launch_dot(dtype, n, x, y, part, out, s), "dot kernel");
    return KPM_OK;
}

kpm_status kpm_dot_noalloc(int32_t dtype, int64_t n, const void* x, const void* y, double* out, void* stream) {
    g_error.clear();
    kpm_status st = blas1_args(dtype, n, {x, y});
    if (st != KPM_OK) return st;
    if (!out) return fail(KPM_EINVAL, "out is NULL");
    // the same two kernels as kpm_dot; their partial sums go to the library's
    // static array on this device (one workgroup's partial per slot: the grid
    // never exceeds naive_dot_partials() workgroups, so every n fits)
    double* part = nullptr;
    KPM_HIP(dot_scratch(&part), "hipGetSymbolAddress(scratch)");
    KPM_HIP(launch_dot(dtype, n, x, y, part, out, static_cast<hipStream_t>(stream)), "dot kernel");
    return KPM_OK;
}

kpm_status kpm_stream(int32_t kind, void* c, const void* a, const void* b, double scalar, int64_t bytes,
                      int32_t wg_per_cu, int32_t nontemporal, void* stream) {
    g_error.clear();
    if (kind != KPM_STREAM_COPY && kind != KPM_STREAM_TRIAD && kind != KPM_STREAM_READ)
        return fail(KPM_EINVAL, "unknown stream kernel");
    if (bytes < 0 || bytes % 16 != 0) return fail(KPM_EINVAL, "bytes must be a non-negative multiple of 16");
    if (wg_per_cu < 1 || wg_per_cu > 32) return fail(KPM_EINVAL, "wg_per_cu must be in [1, 32]");
    if (bytes == 0) return KPM_OK;
    const bool triad = kind == KPM_STREAM_TRIAD;
    if (!c || !a || (triad && !b)) return fail(KPM_EINVAL, "NULL array");
    for (const void* p : {static_cast<const void*>(c), a, triad ? b : a})
        if (reinterpret_cast<uintptr_t>(p) % 16 != 0) return fail(KPM_EINVAL, "arrays must be 16-byte aligned");
    const char* cc = static_cast<const char*>(c);
    // the read kernel writes one double per workgroup, the others `bytes`
    const int64_t c_bytes = kind == KPM_STREAM_READ ? static_cast<int64_t>(device_cus()) * wg_per_cu * 8 : bytes;
    auto overlap = [&](const void* x) {
        const char* xc = static_cast<const char*>(x);
        return xc < cc + c_bytes && cc < xc + bytes;
    };
    if (overlap(a) || (triad && overlap(b))) return fail(KPM_EINVAL, "c overlaps an input");
    KPM_HIP(launch_stream(kind, nontemporal ? 1 : 0, c, a, b, scalar, bytes / 16, wg_per_cu,
                          static_cast<hipStream_t>(stream)),
            "stream kernel");
    return KPM_OK;
}

kpm_status kpm_site_block(void* V, int64_t N, int32_t R, const int64_t* rows, int32_t dtype, void* stream) {
    g_error.clear();
    if (!V || !rows) return fail(KPM_EINVAL, "V or rows is NULL");
    if (dtype != KPM_C128 && dtype != KPM_C64) return fail(KPM_EINVAL, "unknown dtype");
    if (N <= 0 || R <= 0 || R > kMaxStartColumns) return fail(KPM_EINVAL, "need N > 0 and 0 < R <= 64");
    for (int r = 0; r < R; ++r)
        if (rows[r] < 0 || rows[r] >= N) return fail(KPM_EINVAL, "row outside [0, N)");
    KPM_HIP(launch_site_block(V, N, R, rows, dtype, static_cast<hipStream_t>(stream)), "site block kernel");
    return KPM_OK;
}

kpm_status kpm_plane_wave_block(void* V, const int32_t* L, int32_t R, const double* k, const int32_t* orbital,
                                int32_t dtype, void* stream) {
    g_error.clear();
    if (!V || !L || !k || !orbital) return fail(KPM_EINVAL, "V, L, k or orbital is NULL");
    if (dtype != KPM_C128 && dtype != KPM_C64) return fail(KPM_EINVAL, "unknown dtype");
    if (R <= 0 || R > kMaxStartColumns) return fail(KPM_EINVAL, "need 0 < R <= 64");
    if (L[0] <= 0 || L[1] <= 0 || L[2] <= 0) return fail(KPM_EINVAL, "lattice side <= 0");
    if (static_cast<int64_t>(L[0]) * L[1] * L[2] > (INT32_MAX / 4)) return fail(KPM_EINVAL, "lattice too large");
    for (int r = 0; r < R; ++r) {
        if (orbital[r] < 0 || orbital[r] > 3) return fail(KPM_EINVAL, "orbital outside [0, 4)");
        for (int j = 0; j < 3; ++j)
            if (!std::isfinite(k[3 * r + j])) return fail(KPM_EINVAL, "momentum not finite");
    }
    const int Li[3] = {L[0], L[1], L[2]};
    KPM_HIP(launch_plane_wave_block(V, Li, R, k, orbital, dtype, static_cast<hipStream_t>(stream)),
            "plane wave kernel");
    return KPM_OK;
}

kpm_status kpm_dos(const double* mu, int32_t R, int32_t M, int32_t kernel, double kparam, double a, double b,
                   const double* E, int32_t K, double* rho, void* stream) {
    g_error.clear();
    if (!mu || !E || !rho) return fail(KPM_EINVAL, "mu, E or rho is NULL");
    if (R <= 0 || M <= 0 || K <= 0) return fail(KPM_EINVAL, "R, M and K must be positive");
    if (!(a > 0.0) || !std::isfinite(a) || !std::isfinite(b)) return fail(KPM_EINVAL, "need finite a > 0 and finite b");
    if (kernel != KPM_JACKSON && kernel != KPM_DIRICHLET && kernel != KPM_LORENTZ)
        return fail(KPM_EINVAL, "unknown kernel");
    if (kernel == KPM_LORENTZ && !(kparam > 0.0)) return fail(KPM_EINVAL, "Lorentz kernel needs kparam > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    KPM_HIP(launch_dos(mu, R, M, kernel, kparam, a, b, E, K, rho, s), "dos kernel");
    return KPM_OK;
}

kpm_status kpm_random_phase_block(void* V, int64_t N, int32_t R, int32_t dtype, uint64_t seed, void* stream) {
    g_error.clear();
    if (!V) return fail(KPM_EINVAL, "V is NULL");
    if (N <= 0 || R <= 0) return fail(KPM_EINVAL, "N and R must be positive");
    if (dtype != KPM_C128 && dtype != KPM_C64) return fail(KPM_EINVAL, "unknown dtype");
    if (N > (INT64_MAX / 64) / R || N * R > (static_cast<int64_t>(INT32_MAX) * 256))
        return fail(KPM_EINVAL, "block too large");
    KPM_HIP(launch_phase_block(V, N, R, dtype, seed, static_cast<hipStream_t>(stream)), "phase block kernel");
    return KPM_OK;
}

kpm_status kpm_dos_batched(const double* mu, int32_t n_inst, int32_t R, int32_t ld, int32_t M, int32_t kernel,
                           double kparam, const double* a, const double* b, const double* E, int32_t K,
                           int32_t masses, double* rho, void* stream) {
    g_error.clear();
    if (!mu || !a || !b || !E || !rho) return fail(KPM_EINVAL, "mu, a, b, E or rho is NULL");
    if (n_inst <= 0 || R <= 0 || M <= 0 || K <= 0 || ld < M) return fail(KPM_EINVAL, "need n_inst, R, M, K > 0 and ld >= M");
    if (n_inst > 65535) return fail(KPM_EINVAL, "at most 65535 instances per call");
    if (kernel != KPM_JACKSON && kernel != KPM_DIRICHLET && kernel != KPM_LORENTZ)
        return fail(KPM_EINVAL, "unknown kernel");
    if (kernel == KPM_LORENTZ && !(kparam > 0.0)) return fail(KPM_EINVAL, "Lorentz kernel needs kparam > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    KPM_HIP(launch_dos_batched(mu, n_inst, R, ld, M, kernel, kparam, a, b, E, K, masses ? 1 : 0, rho, s),
            "dos kernel");
    return KPM_OK;
}

kpm_status kpm_moment_features(const double* mu, int32_t n_inst, int32_t R, int32_t ld, int32_t n_mom,
                               const float* extra, float* x, void* stream) {
    g_error.clear();
    if (!mu || !x) return fail(KPM_EINVAL, "mu or x is NULL");
    if (n_inst <= 0 || R <= 0 || n_mom <= 0 || ld < n_mom) return fail(KPM_EINVAL, "need n_inst, R, n_mom > 0 and ld >= n_mom");
    hipStream_t s = static_cast<hipStream_t>(stream);
    KPM_HIP(launch_features(mu, n_inst, R, ld, n_mom, extra, x, s), "features kernel");
    return KPM_OK;
}

kpm_status kpm_set_sweep_tuning(const kpm_sweep_tuning* t) {
    g_error.clear();
    if (!t) {
        set_tuning(default_tuning());
        return KPM_OK;
    }
    const kpm_status st = check_tuning(*t);
    if (st != KPM_OK) return st;
    set_tuning(*t);
    return KPM_OK;
}

kpm_status kpm_get_sweep_tuning(kpm_sweep_tuning* t) {
    g_error.clear();
    if (!t) return fail(KPM_EINVAL, "tuning is NULL");
    *t = get_tuning();
    return KPM_OK;
}

kpm_status kpm_sweep_kernel(const kpm_hamiltonian* Hc, int32_t R, int32_t* kernel) {
    g_error.clear();
    if (!Hc || !kernel) return fail(KPM_EINVAL, "H or kernel is NULL");
    TuningScope scope(nullptr);
    *kernel = sweep_kind(Hc, R);
    return KPM_OK;
}

kpm_status kpm_sweep_plan(const kpm_hamiltonian* Hc, int32_t R, const kpm_sweep_tuning* tuning,
                          kpm_sweep_plan_info* out) {
    g_error.clear();
    if (!Hc || !out) return fail(KPM_EINVAL, "H or out is NULL");
    if (!r_supported(R)) return fail(KPM_ENOTSUP, "R must be one of 1, 2, 4, 8, 16, 32, 64");
    kpm_status st;
    if (tuning && (st = check_tuning(*tuning)) != KPM_OK) return st;
    TuningScope scope(tuning);
    const int G = default_group(Hc, R, true);
    const bool lat = use_lattice(Hc, G);
    out->kernel = sweep_kind(Hc, G);
    out->grid = launch_grid(Hc, G);
    out->tile_order = lat ? lattice_order(Hc, out->grid) : -1;
    out->pieces = lat ? lattice_pieces(Hc, G, out->grid, get_tuning().prefetch) : -1;
    out->halves = lat ? G / 32 : -1;
    out->group = G;
    return KPM_OK;
}

kpm_status kpm_sweep_profile_enable(int32_t enable) {
    g_error.clear();
    if (enable < 0) return fail(KPM_EINVAL, "sweep profile period must be >= 0");
    std::lock_guard<std::mutex> g(g_prof.lock);
    g_prof.period = enable;
    g_prof.seen = 0;
    return KPM_OK;
}

kpm_status kpm_sweep_profile_read(int64_t* count, double* total_ms, double* min_ms, double* max_ms) {
    g_error.clear();
    std::lock_guard<std::mutex> g(g_prof.lock);
    double tot = 0.0, lo = 0.0, hi = 0.0;
    for (size_t i = 0; i < g_prof.used; ++i) {
        KPM_HIP(hipEventSynchronize(g_prof.stop[i]), "hipEventSynchronize");
        float ms = 0.0f;
        KPM_HIP(hipEventElapsedTime(&ms, g_prof.start[i], g_prof.stop[i]), "hipEventElapsedTime");
        tot += ms;
        lo = (i == 0 || ms < lo) ? ms : lo;
        hi = (i == 0 || ms > hi) ? ms : hi;
    }
    if (count) *count = static_cast<int64_t>(g_prof.used);
    if (total_ms) *total_ms = tot;
    if (min_ms) *min_ms = lo;
    if (max_ms) *max_ms = hi;
    g_prof.used = 0;
    return KPM_OK;
}

kpm_status kpm_set_batch_tuning(const kpm_batch_tuning* t) {
    g_error.clear();
    if (!t) {
        std::lock_guard<std::mutex> g(g_batch_lock);
        g_batch_tuning = kDefaultBatchTuning;
        return KPM_OK;
    }
    if (t->waves != 0 && t->waves != 4 && t->waves != 8 && t->waves != 16)
        return fail(KPM_EINVAL, "waves must be 0, 4, 8 or 16");
    if (t->wg_per_cu < 0 || t->wg_per_cu > 16) return fail(KPM_EINVAL, "wg_per_cu must be in [0, 16]");
    if (t->dynamic < 0) return fail(KPM_EINVAL, "dynamic must be >= 0");
    if (t->slab < 0) return fail(KPM_EINVAL, "slab must be >= 0");
    std::lock_guard<std::mutex> g(g_batch_lock);
    g_batch_tuning = *t;
    return KPM_OK;
}

kpm_status kpm_get_batch_tuning(kpm_batch_tuning* t) {
    g_error.clear();
    if (!t) return fail(KPM_EINVAL, "tuning is NULL");
    *t = batch_tuning();
    return KPM_OK;
}

kpm_status kpm_moments_batched(const kpm_hamiltonian* const* H, const void* const* V0, int32_t n_inst, int32_t R,
                               int32_t M, double* mu, int32_t flags, void* stream) {
    g_error.clear();
    if (!H || !V0 || !mu) return fail(KPM_EINVAL, "H, V0 or mu is NULL");
    if (n_inst <= 0) return fail(KPM_EINVAL, "n_inst must be positive");
    if (!r_supported(R)) return fail(KPM_ENOTSUP, "R must be one of 1, 2, 4, 8, 16, 32, 64");
    if (M < 2 || (M % 2) != 0) return fail(KPM_EINVAL, "M must be even and >= 2");
    if ((flags & ~(KPM_BATCH_CHECK | KPM_BATCH_GRAPH)) != 0) return fail(KPM_EINVAL, "unknown flag");
    if (static_cast<int64_t>(R) * M > (INT32_MAX / 2)) return fail(KPM_EINVAL, "R * M too large");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(KPM_EDEVICE, "hipGetDevice failed");
    int dtype = -1;
    for (int i = 0; i < n_inst; ++i) {
        if (!H[i] || !V0[i]) return fail(KPM_EINVAL, "H[i] or V0[i] is NULL (i = " + std::to_string(i) + ")");
        if (H[i]->device != dev) return fail(KPM_EINVAL, "H[i] was built on another device");
        if (i == 0) dtype = H[i]->dtype;
        if (H[i]->dtype != dtype) return fail(KPM_EINVAL, "all instances must have one dtype");
        if (H[i]->sell.C > 0)
            return fail(KPM_ENOTSUP, "the batched solver derives its columns from a lattice; H[i] is an imported matrix");
        const uint64_t pair = 2 * real_size(dtype);
        const uint64_t n = static_cast<uint64_t>(H[i]->nrows);
        // 32-bit buffer offsets, with room for the read-ahead past the last pass
        const uint64_t lim = (1ull << 32) - (1ull << 24);
        if (n * R * pair >= lim || n * kWidth * pair >= lim)
            return fail(KPM_ENOTSUP, "an instance's vector block or matrix reaches 4 GiB");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    BatchState& b = *batch_state(dev, s);
    const kpm_batch_tuning bt = batch_tuning();
    const size_t rs = real_size(dtype);

    // instance table: two work blocks and the sweep products per instance
    std::vector<size_t> voff(n_inst);
    size_t vtotal = 0;
    for (int i = 0; i < n_inst; ++i) {
        voff[i] = vtotal;
        const size_t blk = (static_cast<size_t>(H[i]->nrows) * 2 * R * rs + 255) / 256 * 256;
        vtotal += 2 * blk;
    }
    const size_t eta_per = static_cast<size_t>(M / 2) * 3 * R;
    const size_t eta_total = eta_per * n_inst * sizeof(double);
    const bool grows = vtotal > b.vec_bytes || eta_total > b.eta_bytes ||
                       n_inst * sizeof(BatchInst) > b.inst_bytes || n_inst * sizeof(int32_t) > b.order_bytes;
    if (grows) drop_graph(b);   // the captured graph points into the buffers being replaced
    kpm_status st;
    if ((st = grow(&b.vec, &b.vec_bytes, vtotal, "hipMalloc(batch blocks)")) != KPM_OK) return st;
    if ((st = grow(&b.eta, &b.eta_bytes, eta_total, "hipMalloc(batch eta)")) != KPM_OK) return st;
    if ((st = grow(&b.inst, &b.inst_bytes, n_inst * sizeof(BatchInst), "hipMalloc(batch table)")) != KPM_OK)
        return st;
    if ((st = grow(&b.order, &b.order_bytes, n_inst * sizeof(int32_t), "hipMalloc(batch order)")) != KPM_OK)
        return st;
    if (!b.ints) KPM_HIP(hipMalloc(&b.ints, 2 * sizeof(int)), "hipMalloc(batch flags)");
    if (!b.flag_host) KPM_HIP(hipHostMalloc(&b.flag_host, sizeof(int)), "hipHostMalloc(batch flag)");

    std::vector<BatchInst> inst(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        const size_t blk = (static_cast<size_t>(H[i]->nrows) * 2 * R * rs + 255) / 256 * 256;
        char* base = static_cast<char*>(b.vec) + voff[i];
        BatchInst& t = inst[i];
        t = BatchInst{};
        t.val = H[i]->val;
        t.v0 = V0[i];
        t.a = base;
        t.b = base + blk;
        t.eta = b.eta + eta_per * i;
        t.mu = mu + static_cast<size_t>(i) * R * M;
        t.nrows = H[i]->nrows;
        t.inv_a = 1.0 / H[i]->a;
        t.shift = H[i]->b / H[i]->a;
        for (int j = 0; j < 3; ++j) t.L[j] = H[i]->L[j];
        t.by_lx.init(static_cast<uint32_t>(H[i]->L[0]));
        t.by_lxy.init(static_cast<uint32_t>(H[i]->L[0]) * static_cast<uint32_t>(H[i]->L[1]));
        if (bt.slab > 0)
            t.geom = SlabGeom::make(H[i]->L[0], H[i]->L[1], H[i]->L[2], bt.slab, batched_rows_per_pass(dtype, R));
    }
    // longest first (greedy longest-processing-time order), ties by index
    std::vector<int32_t> order(n_inst);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return H[x]->nrows > H[y]->nrows; });

    const int max_w = batched_max_waves(dtype, R);
    if (max_w == 0) return fail(KPM_EINTERNAL, "no batched kernel for this dtype and R");
    // 8 waves (one workgroup per CU, two waves per SIMD) by default: one wave
    // per SIMD leaves the integer work of the gather offsets exposed, and 16
    // waves measured slower on the 512-instance family
    int waves = bt.waves > 0 ? bt.waves : (max_w < 8 ? max_w : 8);
    if (waves > max_w) waves = max_w;
    const int per_cu = bt.wg_per_cu > 0 ? bt.wg_per_cu : 1;
    int grid = device_cus() * per_cu;
    if (grid > n_inst) grid = n_inst;
    const int dynamic = bt.dynamic ? 1 : 0;
    BatchArgs args{b.inst, b.order, n_inst, b.ints, b.ints + 1, M, grid, waves, dynamic, bt.slab};

    const bool use_graph = (flags & KPM_BATCH_GRAPH) != 0;
    bool hit = use_graph && b.exec && b.key_dtype == dtype && b.key_R == R && b.key_M == M &&
               b.key_grid == grid && b.key_waves == waves && b.key_dynamic == dynamic &&
               b.key_slab == bt.slab &&
               b.key_inst.size() == inst.size() && b.key_order == order;
    for (size_t i = 0; hit && i < inst.size(); ++i) hit = same_inst(b.key_inst[i], inst[i]);

    if (hit) {
        KPM_HIP(hipGraphLaunch(b.exec, s), "hipGraphLaunch");
    } else {
        drop_graph(b);
        KPM_HIP(hipMemcpyAsync(b.inst, inst.data(), n_inst * sizeof(BatchInst), hipMemcpyHostToDevice, s),
                "copy instance table");
        KPM_HIP(hipMemcpyAsync(b.order, order.data(), n_inst * sizeof(int32_t), hipMemcpyHostToDevice, s),
                "copy instance order");
        KPM_HIP(hipStreamSynchronize(s), "synchronise");   // the host tables are about to go away
        if (use_graph) {
            if (!b.capture) KPM_HIP(hipStreamCreateWithFlags(&b.capture, hipStreamNonBlocking), "hipStreamCreate");
            KPM_HIP(hipStreamBeginCapture(b.capture, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            hipError_t e1 = launch_zero_ints(b.ints, 2, b.capture);
            hipError_t e2 = e1 == hipSuccess ? launch_batched(dtype, R, args, b.capture) : e1;
            hipGraph_t g = nullptr;
            hipError_t e3 = hipStreamEndCapture(b.capture, &g);
            if (e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return hip_fail(e2, "batched kernel (capture)");
            }
            if (e3 != hipSuccess) return hip_fail(e3, "hipStreamEndCapture");
            b.graph = g;
            KPM_HIP(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0), "hipGraphInstantiate");
            b.key_inst = inst;
            b.key_order = order;
            b.key_dtype = dtype;
            b.key_R = R;
            b.key_M = M;
            b.key_grid = grid;
            b.key_waves = waves;
            b.key_dynamic = dynamic;
            b.key_slab = bt.slab;
            KPM_HIP(hipGraphLaunch(b.exec, s), "hipGraphLaunch");
        } else {
            KPM_HIP(launch_zero_ints(b.ints, 2, s), "zero kernel");
            KPM_HIP(launch_batched(dtype, R, args, s), "batched kernel");
        }
    }
    if (flags & KPM_BATCH_CHECK) {
        KPM_HIP(hipMemcpyAsync(b.flag_host, b.ints + 1, sizeof(int), hipMemcpyDeviceToHost, s), "copy flag");
        KPM_HIP(hipStreamSynchronize(s), "synchronise");
        if (*b.flag_host)
            return fail(KPM_ESPECTRUM, "moments left [-mu_0, mu_0] in at least one instance");
    }
    return KPM_OK;
}

}  // extern "C"

// libmcf host runtime: instance setup, device buffers, the iteration driver and
// the C ABI declared in include/mcf.h.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "mcf.h"
#include "mcf_internal.h"

using namespace mcf;

namespace {

constexpr int MAX_N = 16384;
// kernel timing brackets the dominant launch of every TIMING_STRIDE-th iteration (a stride
// prime to check_every and k_adapt samples the same mix of iteration kinds)
constexpr long long TIMING_STRIDE = 7;
constexpr size_t MAX_GRAPHS = 32;  // captured block shapes kept per handle
constexpr size_t ALIGN = 256;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Pinned host mirrors of the device scalars (three records per handle) come from a process-wide
// free list, allocated in chunks and kept until the process ends: creating and destroying
// handles then calls neither hipHostMalloc nor hipHostFree, which may wait for the whole device
// (a serving loop creates and destroys handles while a pool step runs on another stream).
constexpr int PIN_CHUNK = 32;
std::mutex g_pin_mu;
std::vector<DevScalars *> g_pin_free;

DevScalars *pinned_get()
{
    std::lock_guard<std::mutex> lock(g_pin_mu);
    if (g_pin_free.empty()) {
        DevScalars *chunk = nullptr;
        if (hipHostMalloc((void **)&chunk, sizeof(DevScalars) * 3 * PIN_CHUNK, hipHostMallocDefault) != hipSuccess)
            return nullptr;
        for (int q = PIN_CHUNK - 1; q >= 0; --q) g_pin_free.push_back(chunk + 3 * q);
    }
    DevScalars *p = g_pin_free.back();
    g_pin_free.pop_back();
    return p;
}

void pinned_put(DevScalars *p)
{
    if (!p) return;
    std::lock_guard<std::mutex> lock(g_pin_mu);
    g_pin_free.push_back(p);
}

long long padded_ld(int n) { return (long long)((n + 63) / 64) * 64; }

int node_blocks(int n, int nb)
{
    return ((n + nb - 1) / nb) * n;
}

PartLayout part_layout(int m, int nb)
{
    PartLayout p;
    long long o = 0;
    p.dF = o; o += m;
    p.e = o; o += m;
    p.sup = o; o += m;
    p.a = o; o += m;
    p.b = o; o += m;
    p.dY = o; o += nb;
    p.p = o; o += nb;
    p.conj = o; o += nb;
    p.rnum = o; o += nb;
    p.rden = o; o += nb;
    p.nonpos = o; o += nb;
    p.yinf = o; o += nb;
    p.red = o; o += (long long)CTRL_NQ * CTRL_GROUPS;
    p.total = o;
    return p;
}

// Byte offsets of every device buffer inside one allocation.
struct Plan {
    size_t F, Fhat, D, Y, W, P, Sout, That, Up, cap, rcp, mu, F2, Y2, mu2, tail, head, out_off, in_off, in_edge, inc_off,
        inc, part, sc, total;
};

bool use_fused(int n, int mode) { return mode == MCF_KERNELS_FUSED || (mode == MCF_KERNELS_AUTO && n <= FUSED_MAX_N); }

Plan make_plan(int n, int m, int precision, bool fused, int node_block)
{
    const size_t es = precision == MCF_FP32 ? 4 : 8;
    const size_t ld = (size_t)padded_ld(n);
    const size_t nm = ld * (size_t)m, nn = ld * (size_t)n;
    const PartLayout pl = part_layout(m, node_blocks(n, node_block));
    Plan p;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    p.F = take(nm * es);
    p.Fhat = take(nm * es);
    p.D = take(nm * es);
    p.Y = take(nn * es);
    p.W = take(nn * es);
    p.P = take(fused ? 0 : nn * es);  // two-phase iteration: P = F A^T and the out-edge sums
    p.Sout = take(fused ? 0 : nn * es);
    p.That = take(nn * 8);
    p.Up = take(nn * 8);
    p.cap = take((size_t)m * 8);
    p.rcp = take((size_t)(n + 1) * 8);
    p.mu = take((size_t)m * 8);
    p.F2 = take(fused ? nm * es : 0);  // ping-pong buffers of the fused iteration
    p.Y2 = take(fused ? nn * es : 0);
    p.mu2 = take(fused ? (size_t)m * 8 : 0);
    p.tail = take((size_t)m * 4);
    p.head = take((size_t)m * 4);
    p.out_off = take((size_t)(n + 1) * 4);
    p.in_off = take((size_t)(n + 1) * 4);
    p.in_edge = take((size_t)(m + IN_EDGE_PAD) * 4);
    p.inc_off = take(fused ? (size_t)(n + 1) * 4 : 0);
    p.inc = take(fused ? (size_t)m * 2 * 8 : 0);
    p.part = take((size_t)pl.total * 8);
    p.sc = take(sizeof(DevScalars));
    p.total = o;
    return p;
}

}  // namespace

struct mcf_solver {
    int n = 0, m = 0, precision = 0;
    mcf_pool *pool = nullptr;  // set while the instance is admitted to a batching pool
    int pool_slot = -1;
    long long ld = 0;
    mcf_options opt{};
    Consts c{};
    PartLayout pl{};
    EdgeShape sh{};
    Plan plan{};
    std::vector<int> perm;  // internal edge -> user edge
    char *base = nullptr;
    bool own_mem = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    DevScalars *hs = nullptr;  // pinned host mirror of the device scalars; hs[1], hs[2] are block snapshots
    DevScalars hs_local[3] = {};  // the mirror of a handle that may not allocate (mcf_solve_static)
    hipEvent_t blk_ev[2] = {nullptr, nullptr};  // completion of the snapshot copies
    int state = MCF_RUNNING;
    long long k = 0;  // PDHG iterations completed (authoritative count)
    // fused mode: iteration k reads buffer set ((k - anchor_k) & 1) ^ anchor_par
    long long anchor_k = 0;
    int anchor_par = 0;
    int parity(long long kk) const { return c.fused ? (int)((kk - anchor_k) & 1) ^ anchor_par : 0; }
    // the current state F^{k-1/2}, Y^k lives in buffer set parity(k)
    size_t cur_F() const { return parity(k) ? plan.F2 : plan.F; }
    size_t cur_Y() const { return parity(k) ? plan.Y2 : plan.Y; }
    double seconds = 0.0;
    // kernel timing of the iteration's main launches (fused, or edge + node)
    bool timing = false;
    std::vector<hipEvent_t> ev;  // pairs (start, stop) recorded during the current drive
    std::vector<long long> ev_iters;  // iterations each pair brackets (indexed by pair)
    // instantiated graphs of whole blocks, keyed by the block's shape (see block_key)
    std::map<std::string, hipGraphExec_t> graphs;
    // asynchronous solve (mcf_solve_async): a host thread runs the block loop; while it runs,
    // mcf_status reads `live` (the record of the latest finished block) under `live_mu`
    std::thread worker;
    std::atomic<bool> busy{false}, cancel{false};
    int async_rc = MCF_OK;
    mutable std::mutex live_mu;
    mcf_result live{};
    size_t ev_used = 0, ev_done = 0;
    double edge_ms = 0.0;
    long long edge_launches = 0;

    template <typename T>
    Bufs<T> bufs() const
    {
        Bufs<T> b;
        b.F = (T *)(base + plan.F);
        b.P = (T *)(base + plan.P);
        b.Sout = (T *)(base + plan.Sout);
        b.Fhat = (T *)(base + plan.Fhat);
        b.D = (T *)(base + plan.D);
        b.Y = (T *)(base + plan.Y);
        b.W = (T *)(base + plan.W);
        b.That = (double *)(base + plan.That);
        b.Up = (double *)(base + plan.Up);
        b.tail = (const int *)(base + plan.tail);
        b.head = (const int *)(base + plan.head);
        b.out_off = (const int *)(base + plan.out_off);
        b.in_off = (const int *)(base + plan.in_off);
        b.in_edge = (const int *)(base + plan.in_edge);
        b.inc_off = (const int *)(base + plan.inc_off);
        b.inc = (const int2 *)(base + plan.inc);
        b.cap = (const double *)(base + plan.cap);
        b.rcp = (const double *)(base + plan.rcp);
        b.mu = (double *)(base + plan.mu);
        b.F2 = (T *)(base + plan.F2);
        b.Y2 = (T *)(base + plan.Y2);
        b.mu2 = (double *)(base + plan.mu2);
        b.part = (double *)(base + plan.part);
        b.sc = (DevScalars *)(base + plan.sc);
        return b;
    }
    DevScalars *dsc() const { return (DevScalars *)(base + plan.sc); }
};

namespace {

int hip_err(hipError_t e) { return e == hipSuccess ? MCF_OK : (e == hipErrorOutOfMemory ? MCF_E_NOMEM : MCF_E_DEVICE); }

#define MCF_TRY(expr)                       \
    do {                                    \
        hipError_t _e = (expr);             \
        if (_e != hipSuccess) return hip_err(_e); \
    } while (0)

// Strong connectivity (Section 1.1 requires a directed path between every pair):
// every node is reached from node 0 along edges and along reversed edges.
bool strongly_connected(int n, int m, const int *tail, const int *head)
{
    for (int dir = 0; dir < 2; ++dir) {
        std::vector<int> off(n + 1, 0), adj(m);
        const int *from = dir == 0 ? tail : head, *to = dir == 0 ? head : tail;
        for (int l = 0; l < m; ++l) off[from[l] + 1]++;
        for (int i = 0; i < n; ++i) off[i + 1] += off[i];
        std::vector<int> pos(off.begin(), off.end() - 1);
        for (int l = 0; l < m; ++l) adj[pos[from[l]]++] = to[l];
        std::vector<char> seen(n, 0);
        std::vector<int> stack{0};
        seen[0] = 1;
        int count = 1;
        while (!stack.empty()) {
            int u = stack.back();
            stack.pop_back();
            for (int k = off[u]; k < off[u + 1]; ++k)
                if (!seen[adj[k]]) {
                    seen[adj[k]] = 1;
                    ++count;
                    stack.push_back(adj[k]);
                }
        }
        if (count != n) return false;
    }
    return true;
}

template <typename T>
int upload_problem(mcf_solver *s, const int *tail, const int *head, const double *cap, const double *w)
{
    const int n = s->n, m = s->m;
    const long long ld = s->ld;
    // internal edge order: sorted by (tail, head, user index); out-edges of a node are contiguous
    std::vector<int> &perm = s->perm;
    perm.resize(m);
    for (int l = 0; l < m; ++l) perm[l] = l;
    std::sort(perm.begin(), perm.end(), [&](int a, int b) {
        if (tail[a] != tail[b]) return tail[a] < tail[b];
        if (head[a] != head[b]) return head[a] < head[b];
        return a < b;
    });
    std::vector<int> t(m), h(m), out_off(n + 1, 0), in_off(n + 1, 0), in_edge(m + IN_EDGE_PAD, 0);
    std::vector<double> c(m);
    for (int e = 0; e < m; ++e) {
        t[e] = tail[perm[e]];
        h[e] = head[perm[e]];
        c[e] = cap[perm[e]];
        out_off[t[e] + 1]++;
        in_off[h[e] + 1]++;
    }
    for (int i = 0; i < n; ++i) {
        out_off[i + 1] += out_off[i];
        in_off[i + 1] += in_off[i];
    }
    std::vector<int> pos(in_off.begin(), in_off.end() - 1);
    for (int e = 0; e < m; ++e) in_edge[pos[h[e]]++] = e;  // ascending internal id within each node
    // eta = 1/sqrt(2 d_max), d_i = in-degree + out-degree = (A A^T)_ii (e-eta, Appendix A)
    int dmax = 0;
    for (int i = 0; i < n; ++i)
        dmax = std::max(dmax, (out_off[i + 1] - out_off[i]) + (in_off[i + 1] - in_off[i]));
    const double eta = 1.0 / std::sqrt(2.0 * (double)dmax);
    // weights, padded columns, iterate precision
    std::vector<T> W((size_t)ld * n, T(0));
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) W[(size_t)j * ld + i] = (i == j) ? T(0) : (T)w[(size_t)j * n + i];
    char *b = s->base;
    const Plan &p = s->plan;
    hipStream_t st = s->stream;
    MCF_TRY(hipMemcpyAsync(b + p.W, W.data(), W.size() * sizeof(T), hipMemcpyHostToDevice, st));
    MCF_TRY(hipMemcpyAsync(b + p.cap, c.data(), m * 8, hipMemcpyHostToDevice, st));
    // 1/k for the multiplier mu = (sum_S q - c)/|S| of the projection (a product, within one
    // rounding of the quotient)
    std::vector<double> rcp(n + 1, 0.0);
    for (int k = 1; k <= n; ++k) rcp[k] = 1.0 / (double)k;
    MCF_TRY(hipMemcpyAsync(b + p.rcp, rcp.data(), (n + 1) * 8, hipMemcpyHostToDevice, st));
    MCF_TRY(hipMemcpyAsync(b + p.tail, t.data(), m * 4, hipMemcpyHostToDevice, st));
    MCF_TRY(hipMemcpyAsync(b + p.head, h.data(), m * 4, hipMemcpyHostToDevice, st));
    MCF_TRY(hipMemcpyAsync(b + p.out_off, out_off.data(), (n + 1) * 4, hipMemcpyHostToDevice, st));
    MCF_TRY(hipMemcpyAsync(b + p.in_off, in_off.data(), (n + 1) * 4, hipMemcpyHostToDevice, st));
    MCF_TRY(hipMemcpyAsync(b + p.in_edge, in_edge.data(), in_edge.size() * 4, hipMemcpyHostToDevice, st));
    // per-node incidence list of the fused iteration: entering edges, then leaving edges
    std::vector<int> inc_off(n + 1, 0);
    std::vector<int2> inc((size_t)2 * m);
    if (s->c.fused) {
        size_t at = 0;
        for (int j = 0; j < n; ++j) {
            inc_off[j] = (int)at;
            for (int k = in_off[j]; k < in_off[j + 1]; ++k) inc[at++] = make_int2(in_edge[k], t[in_edge[k]]);
            for (int e = out_off[j]; e < out_off[j + 1]; ++e) inc[at++] = make_int2(e, (int)(h[e] | 0x80000000u));
        }
        inc_off[n] = (int)at;
        MCF_TRY(hipMemcpyAsync(b + p.inc_off, inc_off.data(), (n + 1) * 4, hipMemcpyHostToDevice, st));
        MCF_TRY(hipMemcpyAsync(b + p.inc, inc.data(), inc.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    }
    MCF_TRY(hipMemsetAsync(b + p.part, 0, (size_t)s->pl.total * 8, st));
    std::memset(s->hs, 0, sizeof(DevScalars));
    s->hs->eta = eta;
    s->hs->stop_enabled = 1;
    MCF_TRY(hipMemcpyAsync(b + p.sc, s->hs, sizeof(DevScalars), hipMemcpyHostToDevice, st));
    MCF_TRY(hipStreamSynchronize(st));  // the host vectors above go out of scope
    return MCF_OK;
}

template <typename T>
int do_reset(mcf_solver *s)
{
    MCF_TRY(launch_init<T>(s->c, s->bufs<T>(), s->opt.omega0, s->stream));
    MCF_TRY(hipMemcpyAsync(s->hs, s->dsc(), sizeof(DevScalars), hipMemcpyDeviceToHost, s->stream));
    MCF_TRY(hipStreamSynchronize(s->stream));
    s->state = MCF_RUNNING;
    s->k = 0;
    s->anchor_k = 0;
    s->anchor_par = 0;
    return MCF_OK;
}

int reset_any(mcf_solver *s) { return s->precision == MCF_FP32 ? do_reset<float>(s) : do_reset<double>(s); }

// Writes the host mirror's control fields to the device (stream idle).
int push_scalars(mcf_solver *s)
{
    MCF_TRY(hipMemcpyAsync(s->dsc(), s->hs, sizeof(DevScalars), hipMemcpyHostToDevice, s->stream));
    return MCF_OK;
}

int pull_scalars(mcf_solver *s)
{
    MCF_TRY(hipMemcpyAsync(s->hs, s->dsc(), sizeof(DevScalars), hipMemcpyDeviceToHost, s->stream));
    MCF_TRY(hipStreamSynchronize(s->stream));
    return MCF_OK;
}

hipEvent_t next_event(mcf_solver *s)
{
    if (s->ev_used == s->ev.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        s->ev.push_back(e);
    }
    if (s->ev_iters.size() <= s->ev_used / 2) s->ev_iters.resize(s->ev_used / 2 + 1);
    s->ev_iters[s->ev_used / 2] = 1;  // a pair brackets one iteration unless set otherwise
    return s->ev[s->ev_used++];
}

// Adds up the bracketed iterations whose events lie in [s->ev_done, upto).
int collect_events(mcf_solver *s, size_t upto)
{
    for (size_t k = s->ev_done; k + 1 < upto; k += 2) {
        float ms = 0.f;
        MCF_TRY(hipEventElapsedTime(&ms, s->ev[k], s->ev[k + 1]));
        s->edge_ms += ms;
        s->edge_launches += s->ev_iters[k / 2];
    }
    s->ev_done = upto;
    return MCF_OK;
}

// Enqueues `count` iterations starting at iteration k0; only the last one is a check
// iteration.  Iterations that adapt omega (k a multiple of k_adapt) or check the residual
// write step-norm partials and end in a control launch; the others are two launches.  Every
// argument depends only on the block's shape (block_key): the control launches advance the
// device's iteration count by the iterations since the previous one, and the device count is
// k0 when the block starts (the previous block ended with a control launch).
template <typename T>
int enqueue_block(mcf_solver *s, long long k0, long long count, bool sample = true)
{
    const Bufs<T> b = s->bufs<T>();
    long long k_ctrl = k0;  // iterations counted on the device so far
    for (long long it = 0; it < count; ++it) {
        const long long k = k0 + it;
        const bool check = it == count - 1;
        const bool adapt = adapts_at(s->c, k);
        const bool partial = check || adapt;
        // timed iterations: the dispatches themselves record the start of the first kernel and
        // the end of the last one of the iteration (no extra packets in the stream)
        hipEvent_t e0 = nullptr, e1 = nullptr;
        const bool timed = sample && s->timing && k % TIMING_STRIDE == 0;
        if (timed) {
            e0 = next_event(s);
            e1 = next_event(s);
            if (!e0 || !e1) return MCF_E_DEVICE;
        }
        if (s->c.fused) {
            MCF_TRY(launch_fused<T>(s->c, b, s->pl, s->sh, s->parity(k), check, partial, s->stream, e0, e1));
        } else {
            MCF_TRY(launch_edge<T>(s->c, b, s->pl, s->sh, check, partial, s->stream, e0, nullptr));
            MCF_TRY(launch_node<T>(s->c, b, s->pl, check, partial, s->stream, nullptr, e1));
        }
        if (check) MCF_TRY(launch_residual<T>(s->c, b, s->pl, s->sh, s->stream));
        if (partial) {
            MCF_TRY(launch_control<T>(s->c, b, s->pl, check, adapt, k + 1 - k_ctrl, s->stream));
            k_ctrl = k + 1;
        }
    }
    return MCF_OK;
}

// What makes two blocks enqueue the same launches with the same arguments: their length, the
// buffer set their first iteration reads (fused mode), and where omega adapts.
std::string block_key(const mcf_solver *s, long long k0, long long count)
{
    std::string key = std::to_string(count) + (s->parity(k0) ? "p" : "e");
    for (long long it = 0; it < count; ++it)
        if (adapts_at(s->c, k0 + it)) key += "," + std::to_string(it);
    return key;
}

// Enqueues a block as one launch of its captured graph: captured on first use, then replayed.
template <typename T>
int enqueue_block_graph(mcf_solver *s, long long k0, long long count)
{
    if (!s->opt.graphs) return enqueue_block<T>(s, k0, count);
    const std::string key = block_key(s, k0, count);
    auto it = s->graphs.find(key);
    // a solve uses two or three block shapes; runs of many different lengths go out directly
    // once the cache holds MAX_GRAPHS of them
    // (with kernel timing on, one pair of events spans the whole drive: no per-iteration events)
    if (it == s->graphs.end() && s->graphs.size() >= MAX_GRAPHS) return enqueue_block<T>(s, k0, count, false);
    if (it == s->graphs.end()) {
        MCF_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue_block<T>(s, k0, count, false);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(s->stream, &g);
        if (rc || ec != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return rc ? rc : MCF_E_DEVICE;
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) return MCF_E_DEVICE;
        it = s->graphs.emplace(key, ex).first;
    }
    MCF_TRY(hipGraphLaunch(it->second, s->stream));
    return MCF_OK;
}

// The solve record of the handle's host state.
void fill_result(const mcf_solver *s, mcf_result *r)
{
    const DevScalars &h = *s->hs;
    std::memset(r, 0, sizeof(*r));
    r->state = s->state;
    r->checked = h.checked;
    r->iters = s->k;
    r->r = h.r;
    r->r_paper = h.r_paper;
    r->rel_primal = h.rel_primal;
    r->rel_dual = h.rel_dual;
    r->rel_gap = h.rel_gap;
    r->rel_kkt = h.rel_kkt;
    r->primal_obj = h.primal_obj;
    r->dual_obj = h.dual_obj;
    r->infeasible_frac = h.infeasible_frac;
    r->omega = h.omega;
    r->alpha = h.alpha;
    r->beta = h.beta;
    r->delta_f = h.dF;
    r->delta_y = h.dY;
    r->seconds = s->seconds;
}

// The iteration driver.  Blocks of check_every iterations end with an asynchronous copy
// of the device scalars into a pinned snapshot slot; two blocks are kept in flight, so the
// device never waits for the host to read a snapshot.  With stop_test the device raises
// `stop` when the stop rule holds at a check, and every launch queued after that returns at
// entry.  Without it, exactly target - k iterations run (divergence still stops).
int drive(mcf_solver *s, long long target, bool stop_test)
{
    struct Pending {
        long long k0, count;
        int slot;
        size_t ev_end;
    };
    auto t0 = std::chrono::steady_clock::now();
    int rc = pull_scalars(s);
    if (rc) return rc;
    if (!stop_test || s->hs->state == MCF_RUNNING) {
        s->hs->stop = s->hs->state == MCF_DIVERGED ? 1 : 0;
        s->hs->stop_enabled = stop_test ? 1 : 0;
        if ((rc = push_scalars(s))) return rc;
    }
    const long long K = std::max(1, s->opt.check_every);
    std::deque<Pending> pend;
    long long k_next = s->k;
    const long long k_start = s->k;
    int slot = 0;
    s->ev_used = s->ev_done = 0;
    bool stopped = s->hs->stop != 0;
    // kernel timing with graphs: one pair of stream events around everything the drive enqueues
    const bool span_timing = s->timing && s->opt.graphs && !stopped;
    if (span_timing) {
        hipEvent_t e0 = next_event(s);
        if (!e0) return MCF_E_DEVICE;
        MCF_TRY(hipEventRecord(e0, s->stream));
    }
    while (!stopped) {
        while (pend.size() < 2 && k_next < target) {
            const long long count = std::min(K, target - k_next);
            rc = s->precision == MCF_FP32 ? enqueue_block_graph<float>(s, k_next, count)
                                          : enqueue_block_graph<double>(s, k_next, count);
            if (rc) return rc;
            MCF_TRY(hipMemcpyAsync(s->hs + 1 + slot, s->dsc(), sizeof(DevScalars), hipMemcpyDeviceToHost,
                                   s->stream));
            MCF_TRY(hipEventRecord(s->blk_ev[slot], s->stream));
            pend.push_back({k_next, count, slot, s->ev_used});
            slot ^= 1;
            k_next += count;
        }
        if (pend.empty()) break;
        const Pending r = pend.front();
        pend.pop_front();
        MCF_TRY(hipEventSynchronize(s->blk_ev[r.slot]));
        *s->hs = s->hs[1 + r.slot];
        if (s->timing && !span_timing && (rc = collect_events(s, r.ev_end))) return rc;
        if (s->hs->stop) {
            s->k = s->hs->k;  // the launches after the stop did nothing
            stopped = true;
        } else {
            s->k = r.k0 + r.count;
        }
        if (s->busy.load(std::memory_order_relaxed)) {
            std::lock_guard<std::mutex> lock(s->live_mu);
            fill_result(s, &s->live);
            s->live.state = MCF_RUNNING;
        }
        if (s->cancel.load(std::memory_order_relaxed)) break;  // the handle is being destroyed
    }
    if (span_timing) {
        hipEvent_t e1 = next_event(s);
        if (!e1) return MCF_E_DEVICE;
        MCF_TRY(hipEventRecord(e1, s->stream));
    }
    MCF_TRY(hipStreamSynchronize(s->stream));  // drain a block queued behind a stop
    if (stopped) s->state = s->hs->state == MCF_DIVERGED ? MCF_DIVERGED : MCF_CONVERGED;
    else s->state = stop_test ? MCF_MAX_ITER : MCF_RUNNING;
    if (span_timing) {
        // the span covers the iterations done (and the few launches queued behind a stop, which
        // return at entry)
        s->ev_iters[0] = s->k - k_start;
        if ((rc = collect_events(s, s->ev_used))) return rc;
    } else if (s->timing && !stopped && (rc = collect_events(s, s->ev_used))) {
        // without graphs, sampled iterations queued behind a stop did no work: they are dropped
        return rc;
    }
    s->ev_used = s->ev_done = 0;
    s->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return MCF_OK;
}

template <typename T>
int download_cols(mcf_solver *s, size_t off, int cols, bool edge_order, double *out)
{
    const int n = s->n;
    const long long ld = s->ld;
    std::vector<T> tmp((size_t)ld * cols);
    MCF_TRY(hipMemcpyAsync(tmp.data(), s->base + off, tmp.size() * sizeof(T), hipMemcpyDeviceToHost, s->stream));
    MCF_TRY(hipStreamSynchronize(s->stream));
    for (int c = 0; c < cols; ++c) {
        const int dst = edge_order ? s->perm[c] : c;
        for (int i = 0; i < n; ++i) out[(size_t)dst * n + i] = (double)tmp[(size_t)c * ld + i];
    }
    return MCF_OK;
}

template <typename T>
int upload_cols(mcf_solver *s, size_t off, int cols, bool edge_order, const double *in)
{
    const int n = s->n;
    const long long ld = s->ld;
    std::vector<T> tmp((size_t)ld * cols, T(0));
    for (int c = 0; c < cols; ++c) {
        const int src = edge_order ? s->perm[c] : c;
        for (int i = 0; i < n; ++i) tmp[(size_t)c * ld + i] = (T)in[(size_t)src * n + i];
    }
    MCF_TRY(hipMemcpyAsync(s->base + off, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, s->stream));
    MCF_TRY(hipStreamSynchronize(s->stream));
    return MCF_OK;
}

int download_any(mcf_solver *s, size_t off, int cols, bool edge_order, double *out)
{
    return s->precision == MCF_FP32 ? download_cols<float>(s, off, cols, edge_order, out)
                                    : download_cols<double>(s, off, cols, edge_order, out);
}

int upload_any(mcf_solver *s, size_t off, int cols, bool edge_order, const double *in)
{
    return s->precision == MCF_FP32 ? upload_cols<float>(s, off, cols, edge_order, in)
                                    : upload_cols<double>(s, off, cols, edge_order, in);
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

void mcf_options_default(mcf_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-4;
    o->max_iter = 100000;
    o->precision = MCF_FP64;
    o->stop_rule = MCF_STOP_REL_KKT;
    o->check_every = 1;
    o->k_adapt = 100;
    o->rho = 1.9;
    o->theta = 0.5;
    o->tau = 1e-5;
    o->omega0 = 1.0;
    o->adapt_until = -1;
    o->device = 0;
    o->graphs = 1;
}

size_t mcf_workspace_bytes(int32_t n, int32_t m, int32_t precision)
{
    if (n < 2 || n > MAX_N || m < 1 || (precision != MCF_FP32 && precision != MCF_FP64)) return 0;
    return make_plan(n, m, precision, use_fused(n, MCF_KERNELS_AUTO),
                     node_block_for(n, precision == MCF_FP32 ? 4 : 8)).total;
}

int32_t mcf_edge_shapes(int32_t precision, int32_t *waves, int32_t *vectors, int32_t cap)
{
    if (precision != MCF_FP32 && precision != MCF_FP64) return 0;
    const EdgeShape *list;
    const int cnt = edge_shape_list(precision == MCF_FP32 ? 4 : 8, &list);
    for (int x = 0; x < cnt && x < cap; ++x) {
        if (waves) waves[x] = list[x].par == 2 ? -1 : list[x].par ? 1 : list[x].wpe;
        if (vectors) vectors[x] = list[x].ept;
    }
    return cnt;
}

const char *mcf_strerror(int code)
{
    switch (code) {
    case MCF_OK: return "ok";
    case MCF_E_ARG: return "invalid argument";
    case MCF_E_GRAPH: return "graph is not strongly connected";
    case MCF_E_NOMEM: return "out of device memory";
    case MCF_E_DEVICE: return "HIP device error";
    case MCF_E_STATE: return "invalid solver state";
    default: return "unknown error";
    }
}

void mcf_destroy(mcf_solver *s)
{
    if (!s) return;
    // an asynchronous solve stops after its current block
    s->cancel.store(true, std::memory_order_relaxed);
    if (s->worker.joinable()) s->worker.join();
    if (s->pool) mcf_pool_retire(s->pool, s->pool_slot);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (auto &g : s->graphs) (void)hipGraphExecDestroy(g.second);
    for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : s->blk_ev)
        if (e) (void)hipEventDestroy(e);
    if (s->own_mem && s->base) (void)hipFree(s->base);
    if (s->hs != s->hs_local) pinned_put(s->hs);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"

namespace {
// Validates a problem and its options and builds the host side of a new solver (sizes, launch
// shape, constants, buffer plan); makes no HIP call.  *out is the new solver on success.
int prepare_solver(int32_t n, int32_t m, const int32_t *tail, const int32_t *head, const double *cap, int32_t utility,
                   double gamma, const double *w, const mcf_options *opt, mcf_solver **out)
{
    if (!out) return MCF_E_ARG;
    *out = nullptr;
    mcf_options o;
    if (opt) o = *opt;
    else mcf_options_default(&o);
    if (n < 2 || n > MAX_N || m < 1 || !tail || !head || !cap || !w) return MCF_E_ARG;
    if (utility != MCF_UTIL_LOG && utility != MCF_UTIL_POWER && utility != MCF_UTIL_ALPHA) return MCF_E_ARG;
    if (utility == MCF_UTIL_POWER && !(gamma > 0.0 && gamma < 1.0)) return MCF_E_ARG;
    if (utility == MCF_UTIL_ALPHA && !(gamma > 0.0 && gamma <= 16.0 && gamma != 1.0)) return MCF_E_ARG;
    if (!(o.tol > 0.0) || (o.precision != MCF_FP32 && o.precision != MCF_FP64)) return MCF_E_ARG;
    if (o.stop_rule != MCF_STOP_REL_KKT && o.stop_rule != MCF_STOP_PAPER) return MCF_E_ARG;
    if (!(o.rho > 0.0 && o.rho < 2.0) || !(o.omega0 > 0.0) || !(o.theta >= 0.0 && o.theta <= 1.0)) return MCF_E_ARG;
    if (o.check_every < 1) o.check_every = 1;
    if (o.kernel_mode < MCF_KERNELS_AUTO || o.kernel_mode > MCF_KERNELS_FUSED) return MCF_E_ARG;
    if (o.kernel_mode == MCF_KERNELS_FUSED && n > FUSED_MAX_N) return MCF_E_ARG;
    const int bytes = o.precision == MCF_FP32 ? 4 : 8;
    EdgeShape shape = edge_shape_for(n, bytes);
    if (o.edge_waves != 0 || o.edge_vectors != 0) {
        const EdgeShape want = o.edge_waves == -1 ? EdgeShape{1, o.edge_vectors, 2}
                                                  : EdgeShape{o.edge_waves, o.edge_vectors, o.edge_waves == 1 ? 1 : 0};
        if (!edge_shape_valid(want, n, bytes)) return MCF_E_ARG;
        shape = want;
    }
    int node_block = node_block_for(n, bytes);
    if (o.node_form < 0 || o.node_form > 2) return MCF_E_ARG;
    if (o.node_block != 0) {
        if (o.node_block != 64 && o.node_block != 256) return MCF_E_ARG;
        node_block = o.node_block;
    }
    for (int l = 0; l < m; ++l) {
        if (tail[l] < 0 || tail[l] >= n || head[l] < 0 || head[l] >= n || tail[l] == head[l]) return MCF_E_ARG;
        if (!(cap[l] > 0.0) || !std::isfinite(cap[l])) return MCF_E_ARG;
    }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            if (i != j) {
                const double x = w[(size_t)j * n + i];
                if (!(x > 0.0) || !std::isfinite(x)) return MCF_E_ARG;
            }
    if (!strongly_connected(n, m, tail, head)) return MCF_E_GRAPH;

    mcf_solver *s = new (std::nothrow) mcf_solver();
    if (!s) return MCF_E_NOMEM;
    s->n = n;
    s->m = m;
    s->precision = o.precision;
    s->opt = o;
    s->ld = padded_ld(n);
    s->sh = shape;
    const bool fused = use_fused(n, o.kernel_mode);
    s->plan = make_plan(n, m, o.precision, fused, node_block);
    s->pl = part_layout(m, node_blocks(n, node_block));
    Consts &c = s->c;
    c.n = n;
    c.m = m;
    c.ld = s->ld;
    c.utility = utility;
    c.gamma = utility == MCF_UTIL_LOG ? 0.0 : gamma;
    // power: c1 = gamma / (1 - gamma) of Section 2.3; alpha-fair: the exponent p = 1 / alpha
    c.c1 = utility == MCF_UTIL_POWER ? gamma / (1.0 - gamma) : utility == MCF_UTIL_ALPHA ? 1.0 / gamma : 0.0;
    c.rho = o.rho;
    c.theta = o.theta;
    c.tau = o.tau;
    c.tol = o.tol;
    c.k_adapt = o.k_adapt;
    c.adapt_until = o.adapt_until;
    c.stop_rule = o.stop_rule;
    c.nblk_node = node_blocks(n, node_block);
    c.node_block = node_block;
    c.fused = fused ? 1 : 0;
    c.edge_par = fused ? 0 : s->sh.par;  // the edge shape is the two-phase iteration's
    c.node_latency = o.node_form == 1 ? 1
                     : o.node_form == 2 ? 0
                     : (long long)n * m * (o.precision == MCF_FP32 ? 4 : 8) <= NODE_LATENCY_BYTES ? 1 : 0;
    // edge quantities are added per tail node (per node in the fused iteration), or per workgroup of
    // the flat edge phase
    c.nep = c.edge_par == 2 ? (m + EDGE_PAR_WAVES - 1) / EDGE_PAR_WAVES : n;
    c.nrp = (m + RES_EDGES - 1) / RES_EDGES;
    c.edge_ept = s->sh.ept;
    c.nnp = fused ? n : c.nblk_node;
    c.f_cached = (long long)n * m * (o.precision == MCF_FP32 ? 4 : 8) <= F_CACHED_BYTES ? 1 : 0;
    *out = s;
    return MCF_OK;
}
}  // namespace

extern "C" {

int mcf_create(int32_t n, int32_t m, const int32_t *tail, const int32_t *head, const double *cap, int32_t utility,
               double gamma, const double *w, const mcf_options *opt, mcf_solver **out)
{
    if (!out) return MCF_E_ARG;
    *out = nullptr;
    mcf_solver *s = nullptr;
    if (int rc0 = prepare_solver(n, m, tail, head, cap, utility, gamma, w, opt, &s)) return rc0;
    const mcf_options &o = s->opt;
    int rc = MCF_OK;
    if (hipSetDevice(o.device) != hipSuccess) rc = MCF_E_DEVICE;
    if (!rc) {
        if (o.stream) {
            s->stream = (hipStream_t)o.stream;
        } else if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess) {
            s->own_stream = true;
        } else {
            rc = MCF_E_DEVICE;
        }
    }
    if (!rc && !(s->hs = pinned_get())) rc = MCF_E_NOMEM;
    for (int q = 0; q < 2 && !rc; ++q)
        if (hipEventCreateWithFlags(&s->blk_ev[q], hipEventDisableTiming) != hipSuccess) rc = MCF_E_DEVICE;
    if (!rc) {
        if (o.workspace) {
            if (o.workspace_bytes < s->plan.total || ((uintptr_t)o.workspace % ALIGN)) rc = MCF_E_ARG;
            else s->base = (char *)o.workspace;
        } else {
            hipError_t e = hipMalloc((void **)&s->base, s->plan.total);
            if (e != hipSuccess) rc = hip_err(e);
            else s->own_mem = true;
        }
    }
    if (!rc) {
        rc = o.precision == MCF_FP32 ? upload_problem<float>(s, tail, head, cap, w)
                                     : upload_problem<double>(s, tail, head, cap, w);
    }
    if (!rc) rc = reset_any(s);
    if (rc) {
        mcf_destroy(s);
        return rc;
    }
    *out = s;
    return MCF_OK;
}

}  // extern "C"

// ------------------------------------------------ the entry point that allocates nothing
// Workspace of mcf_solve_static: a file-scope device array, one per GPU, held until the process
// ends.  In host code its name is a host-side stand-in, never a device address: host code uses
// only the address hipGetSymbolAddress returns for the current device (scratch_base).
static __device__ __align__(256) char scratch[MCF_STATIC_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_static_mu[MAX_DEVICES];   // one call at a time per GPU within this process
char *g_static_base[MAX_DEVICES] = {};

// The device address of this GPU's scratch array, looked up once per device with the device
// current (called with g_static_mu[device] held).
int scratch_base(int device, char **out)
{
    if (!g_static_base[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MCF_E_DEVICE;
        g_static_base[device] = (char *)ptr;
    }
    *out = g_static_base[device];
    return MCF_OK;
}

// The block loop of mcf_solve without graphs, events or pinned memory: each block of
// check_every iterations is launched directly, then its scalar record is copied to the host
// and waited for.
int drive_sync(mcf_solver *s)
{
    int rc = pull_scalars(s);
    if (rc) return rc;
    s->hs->stop = 0;
    s->hs->stop_enabled = 1;
    if ((rc = push_scalars(s))) return rc;
    const long long K = std::max(1, s->opt.check_every), target = s->opt.max_iter;
    auto t0 = std::chrono::steady_clock::now();
    bool stopped = false;
    while (!stopped && s->k < target) {
        const long long count = std::min(K, target - s->k);
        rc = s->precision == MCF_FP32 ? enqueue_block<float>(s, s->k, count, false)
                                      : enqueue_block<double>(s, s->k, count, false);
        if (rc) return rc;
        if ((rc = pull_scalars(s))) return rc;
        if (s->hs->stop) {
            s->k = s->hs->k;
            stopped = true;
        } else {
            s->k += count;
        }
    }
    if (stopped) s->state = s->hs->state == MCF_DIVERGED ? MCF_DIVERGED : MCF_CONVERGED;
    else s->state = MCF_MAX_ITER;
    s->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return MCF_OK;
}
}  // namespace

extern "C" {

int mcf_solve_static(int32_t n, int32_t m, const int32_t *tail, const int32_t *head, const double *cap,
                     int32_t utility, double gamma, const double *w, const mcf_options *opt, double *F, double *T,
                     double *Y, mcf_result *result)
{
    if (!result) return MCF_E_ARG;
    if (opt && (opt->workspace || opt->workspace_bytes)) return MCF_E_ARG;  // the static array is the workspace
    mcf_solver *s = nullptr;
    if (int rc0 = prepare_solver(n, m, tail, head, cap, utility, gamma, w, opt, &s)) return rc0;
    const mcf_options &o = s->opt;
    if (s->plan.total > MCF_STATIC_BYTES || o.device < 0 || o.device >= MAX_DEVICES) {
        delete s;
        return MCF_E_ARG;
    }
    std::lock_guard<std::mutex> lock(g_static_mu[o.device]);
    int rc = hipSetDevice(o.device) == hipSuccess ? MCF_OK : MCF_E_DEVICE;
    if (!rc) rc = scratch_base(o.device, &s->base);
    if (!rc) {
        s->hs = s->hs_local;
        s->stream = (hipStream_t)o.stream;  // the caller's stream, or the null stream
        // upload and reset write every buffer the iteration reads before it reads it (the
        // previous call's contents are never used)
        rc = o.precision == MCF_FP32 ? upload_problem<float>(s, tail, head, cap, w)
                                     : upload_problem<double>(s, tail, head, cap, w);
    }
    if (!rc) rc = reset_any(s);
    if (!rc) rc = drive_sync(s);
    if (!rc && F) rc = download_any(s, s->plan.Fhat, s->m, true, F);
    if (!rc && T) rc = download_cols<double>(s, s->plan.That, s->n, false, T);
    if (!rc && Y) rc = download_any(s, s->cur_Y(), s->n, false, Y);
    if (!rc) fill_result(s, result);
    (void)hipStreamSynchronize(s->stream);
    s->stream = nullptr;
    s->base = nullptr;
    mcf_destroy(s);
    return rc;
}

namespace {
// Calls that use the handle wait for nothing: while an asynchronous solve runs they return
// MCF_E_STATE; after it, its thread is joined first.
int idle(mcf_solver *s)
{
    if (s->busy.load(std::memory_order_acquire)) return MCF_E_STATE;
    if (s->worker.joinable()) s->worker.join();
    return MCF_OK;
}
}  // namespace

int mcf_reset(mcf_solver *s)
{
    if (!s) return MCF_E_ARG;
    if (int rc_ = idle(s)) return rc_;
    if (s->pool) return MCF_E_STATE;
    return reset_any(s);
}

int mcf_solve(mcf_solver *s)
{
    if (!s) return MCF_E_ARG;
    if (int rc_ = idle(s)) return rc_;
    if (s->pool) return MCF_E_STATE;
    return drive(s, s->opt.max_iter, true);
}

int mcf_solve_async(mcf_solver *s)
{
    if (!s) return MCF_E_ARG;
    if (int rc = idle(s)) return rc;
    if (s->pool) return MCF_E_STATE;
    {
        std::lock_guard<std::mutex> lock(s->live_mu);
        fill_result(s, &s->live);
        s->live.state = MCF_RUNNING;
    }
    s->async_rc = MCF_OK;
    s->busy.store(true, std::memory_order_release);
    try {
        s->worker = std::thread([s] {
            // the current device is per host thread
            int rc = hipSetDevice(s->opt.device) == hipSuccess ? MCF_OK : MCF_E_DEVICE;
            if (!rc) rc = drive(s, s->opt.max_iter, true);
            s->async_rc = rc;
            s->busy.store(false, std::memory_order_release);
        });
    } catch (...) {
        s->busy.store(false, std::memory_order_release);
        return MCF_E_NOMEM;
    }
    return MCF_OK;
}

int mcf_run(mcf_solver *s, int64_t iters)
{
    if (!s || iters < 0) return MCF_E_ARG;
    if (int rc_ = idle(s)) return rc_;
    if (s->pool) return MCF_E_STATE;
    int rc = pull_scalars(s);
    if (rc) return rc;
    if (s->hs->state == MCF_CONVERGED) {  // run on past a met stop rule
        s->hs->state = MCF_RUNNING;
        s->hs->stop = 0;
        if ((rc = push_scalars(s))) return rc;
    }
    return drive(s, s->k + iters, false);
}

int mcf_status(const mcf_solver *s, mcf_result *r)
{
    if (!s || !r) return MCF_E_ARG;
    if (s->busy.load(std::memory_order_acquire)) {
        std::lock_guard<std::mutex> lock(s->live_mu);
        *r = s->live;
        return MCF_OK;
    }
    fill_result(s, r);
    return s->async_rc;
}

int mcf_get_solution(mcf_solver *s, double *F, double *T, double *Y)
{
    if (!s) return MCF_E_ARG;
    if (int rc_ = idle(s)) return rc_;
    if (s->pool) return MCF_E_STATE;
    int rc = MCF_OK;
    if (F && (rc = download_any(s, s->plan.Fhat, s->m, true, F))) return rc;
    if (T && (rc = download_cols<double>(s, s->plan.That, s->n, false, T))) return rc;
    if (Y && (rc = download_any(s, s->cur_Y(), s->n, false, Y))) return rc;
    return MCF_OK;
}

int mcf_get_state(mcf_solver *s, double *F, double *Y, mcf_scalars *sc)
{
    if (!s) return MCF_E_ARG;
    if (int rc_ = idle(s)) return rc_;
    if (s->pool) return MCF_E_STATE;
    int rc = MCF_OK;
    if (F && (rc = download_any(s, s->cur_F(), s->m, true, F))) return rc;
    if (Y && (rc = download_any(s, s->cur_Y(), s->n, false, Y))) return rc;
    if (sc) {
        if ((rc = pull_scalars(s))) return rc;
        sc->k = s->k;
        sc->omega = s->hs->omega;
        sc->alpha = s->hs->alpha;
        sc->beta = s->hs->beta;
        sc->r = s->hs->r;
    }
    return MCF_OK;
}

int mcf_set_state(mcf_solver *s, const double *F, const double *Y, const mcf_scalars *sc)
{
    if (!s || !F) return MCF_E_ARG;
    if (int rc_ = idle(s)) return rc_;
    if (s->pool) return MCF_E_STATE;
    if (sc && (!(sc->omega > 0.0) || sc->k < 0)) return MCF_E_ARG;
    // the uploaded state becomes buffer set 0 at iteration k (fused mode)
    if (s->c.fused && s->parity(s->k) == 1 && !Y) {
        // keep the current Y: copy it into set 0 first
        MCF_TRY(hipMemcpyAsync(s->base + s->plan.Y, s->base + s->plan.Y2, (size_t)s->ld * s->n *
                               (s->precision == MCF_FP32 ? 4 : 8), hipMemcpyDeviceToDevice, s->stream));
        MCF_TRY(hipMemcpyAsync(s->base + s->plan.mu, s->base + s->plan.mu2, (size_t)s->m * 8,
                               hipMemcpyDeviceToDevice, s->stream));
    } else if (s->c.fused && s->parity(s->k) == 1) {
        MCF_TRY(hipMemcpyAsync(s->base + s->plan.mu, s->base + s->plan.mu2, (size_t)s->m * 8,
                               hipMemcpyDeviceToDevice, s->stream));
    }
    int rc = upload_any(s, s->plan.F, s->m, true, F);
    if (!rc && Y) rc = upload_any(s, s->plan.Y, s->n, false, Y);
    if (rc) return rc;
    if (!s->c.fused) {
        // the two-phase iteration carries P = F A^T of the current F
        MCF_TRY(s->precision == MCF_FP32 ? launch_p_from_f<float>(s->c, s->bufs<float>(), s->stream)
                                         : launch_p_from_f<double>(s->c, s->bufs<double>(), s->stream));
    }
    if ((rc = pull_scalars(s))) return rc;
    if (sc) s->k = sc->k;
    s->anchor_k = s->k;
    s->anchor_par = 0;
    if (sc) {
        s->hs->k = sc->k;
        s->hs->omega = sc->omega;
        s->hs->alpha = s->hs->eta / sc->omega;
        s->hs->beta = s->hs->eta * sc->omega;
    }
    s->hs->stop = 0;
    s->hs->state = MCF_RUNNING;
    s->hs->checked = 0;
    s->state = MCF_RUNNING;
    if ((rc = push_scalars(s))) return rc;
    MCF_TRY(hipStreamSynchronize(s->stream));
    return MCF_OK;
}

int mcf_debug_poison(mcf_solver *s, int32_t which, int64_t index)
{
    if (!s || (which != 0 && which != 1)) return MCF_E_ARG;
    if (int rc_ = idle(s)) return rc_;
    if (s->pool) return MCF_E_STATE;
    const int n = s->n;
    const long long cols = which == 0 ? s->m : n;
    if (index < 0 || index >= cols * n) return MCF_E_ARG;
    long long col = index / n, i = index % n;
    if (which == 0) {
        // user edge -> internal column
        long long internal = -1;
        for (int e = 0; e < s->m; ++e)
            if (s->perm[e] == col) internal = e;
        col = internal;
    }
    const long long off = col * s->ld + i;
    hipError_t e;
    if (s->precision == MCF_FP32) {
        Bufs<float> b = s->bufs<float>();
        if (s->parity(s->k)) { b.F = b.F2; b.Y = b.Y2; }
        e = launch_poison<float>(b, which, off, s->stream);
    } else {
        Bufs<double> b = s->bufs<double>();
        if (s->parity(s->k)) { b.F = b.F2; b.Y = b.Y2; }
        e = launch_poison<double>(b, which, off, s->stream);
    }
    MCF_TRY(e);
    MCF_TRY(hipStreamSynchronize(s->stream));
    return MCF_OK;
}

int mcf_enable_kernel_timing(mcf_solver *s, int32_t enable)
{
    if (!s) return MCF_E_ARG;
    if (int rc_ = idle(s)) return rc_;
    s->timing = enable != 0;
    s->ev_used = s->ev_done = 0;
    s->edge_ms = 0.0;
    s->edge_launches = 0;
    return MCF_OK;
}

int mcf_kernel_time(mcf_solver *s, double *edge_ms, int64_t *edge_launches)
{
    if (!s) return MCF_E_ARG;
    if (int rc_ = idle(s)) return rc_;
    if (edge_ms) *edge_ms = s->edge_ms;
    if (edge_launches) *edge_launches = s->edge_launches;
    return MCF_OK;
}

int mcf_layout(const mcf_solver *s, int32_t *ld, int32_t *edge_block, int32_t *edge_ept, int32_t *kernel_mode)
{
    if (!s) return MCF_E_ARG;
    if (ld) *ld = (int32_t)s->ld;
    if (edge_block) *edge_block = 64 * (s->sh.par ? EDGE_PAR_WAVES : s->sh.wpe);
    if (edge_ept) *edge_ept = s->sh.ept * (s->precision == MCF_FP32 ? 4 : 2);
    if (kernel_mode) *kernel_mode = s->c.fused ? MCF_KERNELS_FUSED : MCF_KERNELS_TWO_PHASE;
    return MCF_OK;
}


// ================================================================ batching pool
}  // extern "C"

struct mcf_pool {
    int device = 0, precision = 0, max_slots = 0, check_every = 1, n_max = FUSED_MAX_N, graphs = 1;
    size_t budget = 0, used = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    PoolShape shape{};
    long long G = 0;  // pool iterations enqueued so far (the device counter equals it when idle)
    std::vector<mcf_solver *> slot;
    std::vector<SlotDesc<double>> desc;  // host copy (the layout does not depend on the iterate type)
    SlotDesc<double> *d_desc = nullptr;
    int2 *d_work = nullptr;
    int2 *d_ework = nullptr, *h_ework = nullptr;  // flat edge items of two-phase slots (device, pinned staging)
    size_t ework_cap = 0;
    int2 *d_nwork = nullptr, *h_nwork = nullptr;  // node items of two-phase slots
    int *d_res_off = nullptr;
    PoolState *d_state = nullptr;
    DevScalars *d_snap = nullptr;
    DevScalars *h_snap = nullptr;         // pinned
    SlotDesc<double> *h_desc = nullptr;   // pinned staging
    int2 *h_work = nullptr;               // pinned staging
    int *h_res_off = nullptr;             // pinned staging
    PoolState *h_state = nullptr;         // pinned staging
    int nwork = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
    // captured steps, keyed by their length, the iterations at which some slot adapts omega and
    // the grids; each with the step count of its last use (least recently used goes first)
    std::map<std::string, std::pair<hipGraphExec_t, long long>> graphs_cache;
    long long steps = 0;
};

namespace {

// A launch grid for `items` work items: the count rounded up to a multiple of an eighth of its
// leading power of two (at least 256), so that the few grids a pool passes through as instances
// come and go are captured once each, at most 1/8 of the workgroups idle.
int pool_grid(int items)
{
    if (items <= 0) return 0;
    int p2 = 1;
    while (p2 * 2 <= items) p2 *= 2;
    const int g = std::max(256, p2 / 8);
    return (items + g - 1) / g * g;
}

int pool_upload(mcf_pool *p)
{
    // the stream is idle here (callers synchronize first), so the staging buffers are free
    std::memcpy(p->h_desc, p->desc.data(), sizeof(SlotDesc<double>) * p->max_slots);
    MCF_TRY(hipMemcpyAsync(p->d_desc, p->h_desc, sizeof(SlotDesc<double>) * p->max_slots, hipMemcpyHostToDevice,
                           p->stream));
    // node items of the largest instances first: their workgroups cost the most, and starting
    // them first leaves the small ones to fill the end of the launch
    std::vector<int> order;
    for (int sl = 0; sl < p->max_slots; ++sl)
        if (p->desc[sl].active) order.push_back(sl);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return p->desc[a].c.n > p->desc[b].c.n; });
    int nw = 0, nres = 0, ne = 0, nn = 0;
    size_t ne_need = 0;
    for (int sl : order)
        if (!p->desc[sl].c.fused) ne_need += p->desc[sl].c.nep;
    if (ne_need > p->ework_cap) {  // grow the edge-item lists (the stream is idle)
        const size_t cap = std::max(ne_need, 2 * p->ework_cap);
        // every graph captured so far holds the old list's address in its kernel arguments
        for (auto &g : p->graphs_cache) (void)hipGraphExecDestroy(g.second.first);
        p->graphs_cache.clear();
        if (p->d_ework) (void)hipFree(p->d_ework);
        if (p->h_ework) (void)hipHostFree(p->h_ework);
        p->d_ework = nullptr;
        p->h_ework = nullptr;
        p->ework_cap = 0;
        MCF_TRY(hipMalloc((void **)&p->d_ework, sizeof(int2) * cap));
        MCF_TRY(hipHostMalloc((void **)&p->h_ework, sizeof(int2) * cap, hipHostMallocDefault));
        p->ework_cap = cap;
    }
    for (int sl : order) {
        const Consts &c = p->desc[sl].c;
        if (c.fused) {
            for (int j = 0; j < c.n; ++j) p->h_work[nw++] = make_int2(sl, j);
        } else {
            for (int blk = 0; blk < c.nep; ++blk) p->h_ework[ne++] = make_int2(sl, blk);
            for (int x = 0; x < c.nblk_node; ++x) p->h_nwork[nn++] = make_int2(sl, x);
        }
    }
    for (int sl = 0; sl < p->max_slots; ++sl) {
        p->h_res_off[sl] = nres;
        if (p->desc[sl].active) nres += p->desc[sl].c.nrp;
    }
    p->h_res_off[p->max_slots] = nres;
    p->nwork = nw + ne;
    p->shape.grid = pool_grid(nw);
    p->shape.res_grid = pool_grid(nres);
    p->shape.edge_grid = pool_grid(ne);
    p->shape.node_grid = pool_grid((nn + POOL_NODE_WAVES - 1) / POOL_NODE_WAVES);
    p->h_state->G = p->G;
    p->h_state->nwork = nw;
    p->h_state->nres = nres;
    p->h_state->nedge = ne;
    p->h_state->nnode = nn;
    if (nw) MCF_TRY(hipMemcpyAsync(p->d_work, p->h_work, sizeof(int2) * nw, hipMemcpyHostToDevice, p->stream));
    if (ne) MCF_TRY(hipMemcpyAsync(p->d_ework, p->h_ework, sizeof(int2) * ne, hipMemcpyHostToDevice, p->stream));
    if (nn) MCF_TRY(hipMemcpyAsync(p->d_nwork, p->h_nwork, sizeof(int2) * nn, hipMemcpyHostToDevice, p->stream));
    MCF_TRY(hipMemcpyAsync(p->d_res_off, p->h_res_off, sizeof(int) * (p->max_slots + 1), hipMemcpyHostToDevice,
                           p->stream));
    MCF_TRY(hipMemcpyAsync(p->d_state, p->h_state, sizeof(PoolState), hipMemcpyHostToDevice, p->stream));
    MCF_TRY(hipStreamSynchronize(p->stream));
    return MCF_OK;
}

// iteration count and state of a slot from the latest snapshot
void pool_refresh(mcf_pool *p, int sl)
{
    mcf_solver *s = p->slot[sl];
    const SlotDesc<double> &d = p->desc[sl];
    *s->hs = p->h_snap[sl];
    long long k = std::min(d.k0 + (p->G - d.G0), (long long)d.max_iter);
    if (s->hs->stop) k = s->hs->k;
    s->k = k;
    s->anchor_k = k;
    s->anchor_par = d.par0 ^ (int)((k - d.k0) & 1);
    if (s->hs->stop) s->state = s->hs->state == MCF_DIVERGED ? MCF_DIVERGED : MCF_CONVERGED;
    else if (k >= d.max_iter) s->state = MCF_MAX_ITER;
    else s->state = MCF_RUNNING;
}

// The step's iterations (offsets from G) at which some active slot adapts omega: they end in a
// control launch.  A slot whose stop flag was raised in the meantime is skipped by the kernels.
std::vector<int> pool_adapt_points(const mcf_pool *p, int iters)
{
    std::vector<int> at;
    for (int it = 0; it < iters; ++it)
        for (int sl = 0; sl < p->max_slots; ++sl) {
            const SlotDesc<double> &d = p->desc[sl];
            if (!d.active) continue;
            const long long k = d.k0 + (p->G + it - d.G0);
            if (k < d.max_iter && adapts_at(d.c, k)) {
                at.push_back(it);
                break;
            }
        }
    return at;
}

// Enqueues one step: `iters` pool iterations (the last one checks every slot), the control
// launches at the adapt points and at the check, and the gather of every slot's record, which
// advances the device's G.  Every argument is fixed for the pool or by the step's key.
template <typename T>
int pool_enqueue(mcf_pool *p, int iters, const std::vector<int> &adapt_at)
{
    const SlotDesc<T> *slots = (const SlotDesc<T> *)p->d_desc;
    size_t a = 0;
    for (int it = 0; it < iters; ++it) {
        const bool check = it == iters - 1;
        const bool adapt = a < adapt_at.size() && adapt_at[a] == it;
        if (adapt) ++a;
        MCF_TRY(launch_pool_iteration<T>(slots, p->d_work, p->d_ework, p->d_nwork, p->d_res_off, p->d_state,
                                         p->max_slots, p->shape, it, check, check || adapt, p->stream));
    }
    MCF_TRY(launch_pool_gather<T>(slots, p->max_slots, p->d_snap, p->d_state, iters, p->stream));
    return MCF_OK;
}

int pool_enqueue_any(mcf_pool *p, int iters, const std::vector<int> &adapt_at)
{
    return p->precision == MCF_FP32 ? pool_enqueue<float>(p, iters, adapt_at) : pool_enqueue<double>(p, iters, adapt_at);
}

// A step as one launch of its captured graph (captured on first use, then replayed), or
// launched directly when graphs are off.  A full cache drops its least recently used graph.
int pool_enqueue_step(mcf_pool *p, int iters)
{
    const std::vector<int> adapt_at = pool_adapt_points(p, iters);
    if (!p->graphs) return pool_enqueue_any(p, iters, adapt_at);
    std::string key = std::to_string(iters) + "g" + std::to_string(p->shape.grid) + "r" +
                      std::to_string(p->shape.res_grid) + "e" + std::to_string(p->shape.edge_grid) + "n" +
                      std::to_string(p->shape.node_grid);
    for (int it : adapt_at) key += "," + std::to_string(it);
    auto g = p->graphs_cache.find(key);
    if (g == p->graphs_cache.end()) {
        if (p->graphs_cache.size() >= MAX_GRAPHS) {  // no step is in flight (mcf_pool_step synced)
            auto lru = p->graphs_cache.begin();
            for (auto q = p->graphs_cache.begin(); q != p->graphs_cache.end(); ++q)
                if (q->second.second < lru->second.second) lru = q;
            (void)hipGraphExecDestroy(lru->second.first);
            p->graphs_cache.erase(lru);
        }
        MCF_TRY(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
        const int rc = pool_enqueue_any(p, iters, adapt_at);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(p->stream, &graph);
        if (rc || ec != hipSuccess || !graph) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc ? rc : MCF_E_DEVICE;
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return MCF_E_DEVICE;
        g = p->graphs_cache.emplace(key, std::make_pair(ex, 0LL)).first;
    }
    g->second.second = ++p->steps;
    MCF_TRY(hipGraphLaunch(g->second.first, p->stream));
    return MCF_OK;
}

}  // namespace

extern "C" {

void mcf_pool_options_default(mcf_pool_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = MCF_FP32;
    o->max_slots = 64;
    o->check_every = 20;
    o->n_max = FUSED_MAX_N;
    o->graphs = 1;
}

int mcf_pool_create(const mcf_pool_options *opt, mcf_pool **out)
{
    if (!out) return MCF_E_ARG;
    *out = nullptr;
    mcf_pool_options o;
    if (opt) o = *opt;
    else mcf_pool_options_default(&o);
    const int bytes = o.precision == MCF_FP32 ? 4 : 8;
    if ((o.precision != MCF_FP32 && o.precision != MCF_FP64) || o.max_slots < 1 || o.max_slots > MCF_POOL_MAX_SLOTS ||
        o.check_every < 1)
        return MCF_E_ARG;
    if (o.n_max == 0) o.n_max = FUSED_MAX_N;
    if (o.n_max < 2 || o.n_max > FUSED_MAX_N) return MCF_E_ARG;
    if (o.waves != 0 && !pool_waves_valid(o.waves, bytes)) return MCF_E_ARG;
    mcf_pool *p = new (std::nothrow) mcf_pool();
    if (!p) return MCF_E_NOMEM;
    p->device = o.device;
    p->precision = o.precision;
    p->budget = o.hbm_budget;
    p->max_slots = o.max_slots;
    p->check_every = o.check_every;
    p->n_max = o.n_max;
    p->graphs = o.graphs ? 1 : 0;
    p->slot.assign(o.max_slots, nullptr);
    p->desc.assign(o.max_slots, SlotDesc<double>{});
    p->shape = pool_shape_for(o.n_max, bytes);
    if (o.waves) p->shape.waves = o.waves;
    int rc = MCF_OK;
    if (hipSetDevice(o.device) != hipSuccess) rc = MCF_E_DEVICE;
    if (!rc) {
        if (o.stream) p->stream = (hipStream_t)o.stream;
        else if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) == hipSuccess) p->own_stream = true;
        else rc = MCF_E_DEVICE;
    }
    const size_t work_cap = (size_t)o.max_slots * FUSED_MAX_N;
    // node items of a two-phase slot: n columns of ceil(n/64) row blocks
    const size_t nwork_cap = (size_t)o.max_slots * FUSED_MAX_N * ((FUSED_MAX_N + 63) / 64);
    if (!rc && (hipMalloc((void **)&p->d_desc, sizeof(SlotDesc<double>) * o.max_slots) != hipSuccess ||
                hipMalloc((void **)&p->d_work, sizeof(int2) * work_cap) != hipSuccess ||
                hipMalloc((void **)&p->d_nwork, sizeof(int2) * nwork_cap) != hipSuccess ||
                hipMalloc((void **)&p->d_res_off, sizeof(int) * (o.max_slots + 1)) != hipSuccess ||
                hipMalloc((void **)&p->d_state, sizeof(PoolState)) != hipSuccess ||
                hipMalloc((void **)&p->d_snap, sizeof(DevScalars) * o.max_slots) != hipSuccess))
        rc = MCF_E_NOMEM;
    if (!rc && (hipHostMalloc((void **)&p->h_snap, sizeof(DevScalars) * o.max_slots, hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc((void **)&p->h_desc, sizeof(SlotDesc<double>) * o.max_slots, hipHostMallocDefault) !=
                    hipSuccess ||
                hipHostMalloc((void **)&p->h_work, sizeof(int2) * work_cap, hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc((void **)&p->h_nwork, sizeof(int2) * nwork_cap, hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc((void **)&p->h_res_off, sizeof(int) * (o.max_slots + 1), hipHostMallocDefault) !=
                    hipSuccess ||
                hipHostMalloc((void **)&p->h_state, sizeof(PoolState), hipHostMallocDefault) != hipSuccess))
        rc = MCF_E_NOMEM;
    if (!rc && hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess) rc = MCF_E_DEVICE;
    if (!rc) rc = pool_upload(p);
    if (rc) {
        mcf_pool_destroy(p);
        return rc;
    }
    *out = p;
    return MCF_OK;
}

void mcf_pool_destroy(mcf_pool *p)
{
    if (!p) return;
    if (p->pending) (void)mcf_pool_sync(p);  // refreshes every slot's state
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    for (int sl = 0; sl < p->max_slots; ++sl)
        if (p->slot[sl]) {
            p->slot[sl]->pool = nullptr;
            p->slot[sl]->pool_slot = -1;
        }
    for (auto &g : p->graphs_cache) (void)hipGraphExecDestroy(g.second.first);
    if (p->done) (void)hipEventDestroy(p->done);
    if (p->d_desc) (void)hipFree(p->d_desc);
    if (p->d_work) (void)hipFree(p->d_work);
    if (p->d_ework) (void)hipFree(p->d_ework);
    if (p->d_nwork) (void)hipFree(p->d_nwork);
    if (p->h_ework) (void)hipHostFree(p->h_ework);
    if (p->h_nwork) (void)hipHostFree(p->h_nwork);
    if (p->d_res_off) (void)hipFree(p->d_res_off);
    if (p->d_state) (void)hipFree(p->d_state);
    if (p->d_snap) (void)hipFree(p->d_snap);
    if (p->h_snap) (void)hipHostFree(p->h_snap);
    if (p->h_desc) (void)hipHostFree(p->h_desc);
    if (p->h_work) (void)hipHostFree(p->h_work);
    if (p->h_res_off) (void)hipHostFree(p->h_res_off);
    if (p->h_state) (void)hipHostFree(p->h_state);
    if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
}

int mcf_pool_admit(mcf_pool *p, mcf_solver *s, int32_t *slot)
{
    if (!p || !s) return MCF_E_ARG;
    if (int rc_ = idle(s)) return rc_;
    if (s->pool || s->precision != p->precision || s->n > p->n_max) return MCF_E_ARG;
    // a two-phase instance must take the flat edge phase (at most 4 vectors per lane) and 64-thread
    // node blocks, the forms the pool's launches run (mcf_pool_instance_options gives them)
    if (!s->c.fused && (s->c.edge_par != 2 || s->c.edge_ept > 4 || s->c.node_block != 64)) return MCF_E_ARG;
    if (s->state == MCF_CONVERGED || s->state == MCF_DIVERGED) return MCF_E_STATE;
    int rc = mcf_pool_sync(p);
    if (rc) return rc;
    if (p->budget && p->used + s->plan.total > p->budget) return MCF_E_NOMEM;
    int sl = -1;
    for (int q = 0; q < p->max_slots && sl < 0; ++q)
        if (!p->slot[q]) sl = q;
    if (sl < 0) return MCF_E_NOMEM;
    MCF_TRY(hipStreamSynchronize(s->stream));
    if ((rc = pull_scalars(s))) return rc;
    s->hs->stop = 0;
    s->hs->state = MCF_RUNNING;
    s->hs->stop_enabled = 1;
    if ((rc = push_scalars(s))) return rc;
    MCF_TRY(hipStreamSynchronize(s->stream));
    SlotDesc<double> &d = p->desc[sl];
    d.c = s->c;
    d.b = s->bufs<double>();  // pointers only: the same layout serves FP32 instances
    d.pl = s->pl;
    d.G0 = p->G;
    d.k0 = s->k;
    d.max_iter = s->opt.max_iter;
    d.par0 = s->parity(s->k);
    d.active = 1;
    p->slot[sl] = s;
    p->used += s->plan.total;
    s->pool = p;
    s->pool_slot = sl;
    s->state = MCF_RUNNING;
    if ((rc = pool_upload(p))) return rc;
    p->h_snap[sl] = *s->hs;
    if (slot) *slot = sl;
    return MCF_OK;
}

int mcf_pool_step(mcf_pool *p, int32_t iters)
{
    if (!p || iters < 1) return MCF_E_ARG;
    int rc = mcf_pool_sync(p);
    if (rc) return rc;
    if (p->nwork == 0) return MCF_OK;
    if ((rc = pool_enqueue_step(p, iters))) return rc;
    p->G += iters;
    MCF_TRY(hipMemcpyAsync(p->h_snap, p->d_snap, sizeof(DevScalars) * p->max_slots, hipMemcpyDeviceToHost, p->stream));
    MCF_TRY(hipEventRecord(p->done, p->stream));
    p->pending = true;
    return MCF_OK;
}

int mcf_pool_sync(mcf_pool *p)
{
    if (!p) return MCF_E_ARG;
    if (!p->pending) return MCF_OK;
    MCF_TRY(hipEventSynchronize(p->done));
    p->pending = false;
    for (int sl = 0; sl < p->max_slots; ++sl)
        if (p->slot[sl]) pool_refresh(p, sl);
    return MCF_OK;
}

int mcf_pool_poll(mcf_pool *p, int32_t slot, mcf_result *out)
{
    if (!p || slot < 0 || slot >= p->max_slots || !p->slot[slot] || !out) return MCF_E_ARG;
    return mcf_status(p->slot[slot], out);
}

int mcf_pool_retire(mcf_pool *p, int32_t slot)
{
    if (!p || slot < 0 || slot >= p->max_slots || !p->slot[slot]) return MCF_E_ARG;
    int rc = mcf_pool_sync(p);
    if (rc) return rc;
    MCF_TRY(hipStreamSynchronize(p->stream));
    mcf_solver *s = p->slot[slot];
    pool_refresh(p, slot);
    p->desc[slot].active = 0;
    p->slot[slot] = nullptr;
    p->used -= s->plan.total;
    s->pool = nullptr;
    s->pool_slot = -1;
    return pool_upload(p);
}

int mcf_pool_instance_options(const mcf_pool *p, int32_t n, mcf_options *o)
{
    if (!p || !o || n < 2 || n > p->n_max) return MCF_E_ARG;
    o->precision = p->precision;
    const int bytes = p->precision == MCF_FP32 ? 4 : 8;
    if (pool_org_for(n, bytes) == 1) {
        const int vec = 16 / bytes;
        o->kernel_mode = MCF_KERNELS_TWO_PHASE;
        o->edge_waves = -1;
        o->edge_vectors = n <= 64 * vec ? 1 : n <= 128 * vec ? 2 : 4;
        o->node_block = 64;
    } else {
        o->kernel_mode = MCF_KERNELS_FUSED;
        o->edge_waves = o->edge_vectors = o->node_block = 0;
    }
    return MCF_OK;
}

int mcf_pool_shape(const mcf_pool *p, int32_t *waves, int32_t *grid, int32_t *max_ept)
{
    if (!p) return MCF_E_ARG;
    if (waves) *waves = p->shape.waves;
    if (grid) *grid = p->shape.grid;
    if (max_ept) *max_ept = p->shape.max_ept;
    return MCF_OK;
}

int mcf_pool_info(const mcf_pool *p, int32_t *active, size_t *used_bytes, int64_t *iterations)
{
    if (!p) return MCF_E_ARG;
    int a = 0;
    for (int sl = 0; sl < p->max_slots; ++sl) a += p->slot[sl] != nullptr;
    if (active) *active = a;
    if (used_bytes) *used_bytes = p->used;
    if (iterations) *iterations = p->G;
    return MCF_OK;
}
}  // extern "C"

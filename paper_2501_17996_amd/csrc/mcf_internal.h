// Internal declarations shared by the libmcf kernels and its host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcf {

// Device-resident scalar state of Algorithm 2.1 and the latest check record.
// The control kernel is the only writer during a solve; the host reads it after
// each block of iterations and writes it only while the stream is idle.
struct DevScalars {
    double omega, alpha, beta, eta;
    double dF, dY;
    double r, r_paper, rel_primal, rel_dual, rel_gap, rel_kkt;
    double primal_obj, dual_obj, infeasible_frac, a, b, e;
    long long k;  // iterations completed as of the last control launch (the host keeps the live count)
    int stop;     // 1: every kernel returns at entry (set on convergence or divergence)
    int state;    // MCF_RUNNING / MCF_CONVERGED / MCF_DIVERGED
    int checked;  // the check fields belong to the last iteration
    int stop_enabled;  // 1: a met stop rule raises `stop` (mcf_solve); 0: run on (mcf_run)
};

// Read-only problem description and constants of one instance.
struct Consts {
    int n, m;
    long long ld;          // padded column length of F, Y, W, T, U'
    int utility;           // 0 log, 1 power
    double gamma, c1, rho, theta, tau, tol;
    int k_adapt, stop_rule;
    long long adapt_until;  // omega adapts only while k < adapt_until (< 0: always)
    int nblk_node;         // node-phase blocks (partials per quantity)
    int node_block;        // threads per node-phase block (64 or 256)
    int fused;             // 1: node-centric single-launch iteration (n <= FUSED_MAX_N)
    int nep, nnp;          // partials per edge quantity (dF, e, sup; one per tail node, or per workgroup of
                           // the flat edge phase) and per node quantity
    int edge_par;          // 1: out-edge sums grouped by wave (concurrent edge phase); 2: flat edge phase
                           // (out-edge sums gathered by the node phase)
    int node_latency;      // 1: regular node launches in the latency form (F within NODE_LATENCY_BYTES)
    int nrp;               // partials of the residual pass (a, b; one per RES_EDGES edges)
    int edge_ept;          // 16-byte vectors per lane of the two-phase edge shape
    int f_cached;          // 1: F within F_CACHED_BYTES, read and written with ordinary accesses by the
                           // one-wave edge phases (else non-temporal)
};

// Algorithm 2.1 step 3 adapts omega at iterations k that are multiples of k_adapt (k = 0
// included), here also limited to k < adapt_until when that is set.
__host__ __device__ inline bool adapts_at(const Consts &c, long long k)
{
    return c.k_adapt > 0 && k % c.k_adapt == 0 && (c.adapt_until < 0 || k < c.adapt_until);
}

// Largest n served by the node-centric fused iteration (one wave per edge column).
constexpr int FUSED_MAX_N = 512;
// Incidence entries of one node staged in LDS at a time by the fused iteration.
constexpr int FUSED_INC_CHUNK = 256;
// Edges (one wave each) per block of the residual pass.
constexpr int RES_EDGES = 16;
// Entries (edge 0) past the end of the device in-edge list, so that the node phase can load a
// whole batch of edge ids at once.
constexpr int IN_EDGE_PAD = 16;
// Largest F (bytes) for which the regular node launch takes its latency form: all of a
// thread's loads in flight at once.  Such an F stays largely in the 256 MB Infinity Cache, where
// latency bounds the launch; beyond it the launch streams from HBM and the form that keeps
// fewer loads in flight per wave is measurably faster (crossover between n = 3000 and 4096 at
// out-degree 10 in FP32).
constexpr long long NODE_LATENCY_BYTES = 512ll << 20;
// Largest F (bytes) that the one-wave edge phases (concurrent and flat, n <= 2048) read and write
// with ordinary loads and stores: an F that fits the Infinity Cache is then still there when the
// node phase gathers it (config3, F = 40 MB: edge launch 20.1 -> 19.5 us, node 19.4 -> 18.8 us).
// Larger ones stream with non-temporal accesses, which leave the caches to Y.
constexpr long long F_CACHED_BYTES = 256ll << 20;

// Offsets (in doubles) of the partial-sum segments.
struct PartLayout {
    long long dF, e, sup, a, b;               // m each (one per edge)
    long long dY, p, conj, rnum, rden, nonpos, yinf;  // nblk_node each
    long long red;                            // CTRL_NQ * CTRL_GROUPS: first-level sums of the control
    long long total;
};

// The control launch reduces CTRL_NQ partial segments.  When the longest one has more than
// CTRL_SPLIT_MIN entries, a first launch of CTRL_GROUPS workgroups sums fixed consecutive ranges
// of every segment (CTRL_GROUPS values each), and the control's single workgroup adds those: a
// single workgroup alone reads config4's 400,000 node partials per quantity in 0.7 ms.
constexpr int CTRL_NQ = 12;
constexpr int CTRL_GROUPS = 256;
constexpr long long CTRL_SPLIT_MIN = 8192;

// Device buffers of one instance.  In fused mode F, Y and mu ping-pong with F2, Y2,
// mu2: iteration k reads the buffers of parity (k + parity offset) & 1 and writes the others.
// The two-phase iteration keeps P = F A^T of the current F (n x n, like Y) and a staging
// column per node, Sout[:, t] = sum of F over the edges leaving t, written by the edge phase.
template <typename T>
struct Bufs {
    T *F, *Fhat, *D, *Y, *W;
    T *P, *Sout;
    T *F2, *Y2;
    double *mu2;
    double *That, *Up;
    const int *tail, *head, *out_off, *in_off, *in_edge;
    // per-node incidence list (fused mode): entries inc_off[j] .. inc_off[j+1] are the edges
    // entering j (in in_edge order) then the edges leaving j, as {edge, other end | 1<<31 if leaving}
    const int *inc_off;
    const int2 *inc;
    const double *cap;
    const double *rcp;     // rcp[k] = 1/k for k = 1..n (support sizes of a projection)
    double *mu;            // per-edge multiplier of the last projection (warm start of the next one)
    double *part;
    DevScalars *sc;
};

// Launch shape of the two-phase edge kernel: `wpe` waves (of 64 lanes) per tail node, which
// project its out-edge columns one after another, and `ept` 16-byte vectors per lane.  With
// wpe == 1 a 256-thread block carries 4 tail nodes, one per wave.
// par == 1: the tail's out-edges are projected concurrently, one wave per edge in an 8-wave
// workgroup (a whole column per wave: n <= 64 * ept * 16 / bytes), and the out-edge sums are
// added per wave and then over the waves in wave order.  par == 2: flat, one wave per edge
// over a grid of 8-edge workgroups, no out-edge sums (the node phase gathers the out-edges).
struct EdgeShape {
    int wpe, ept, par;
};
// Waves per workgroup of the concurrent edge phase.
constexpr int EDGE_PAR_WAVES = 8;
EdgeShape edge_shape_for(int n, int bytes);
// the compiled two-phase edge shapes for iterate size `bytes`; whether `sh` is one of them and
// its columns hold n entries
int edge_shape_list(int bytes, const EdgeShape **list);
bool edge_shape_valid(EdgeShape sh, int n, int bytes);

// Kernel launchers (defined in mcf_kernels.hip).
template <typename T>
hipError_t launch_init(const Consts &c, const Bufs<T> &b, double omega0, hipStream_t st);
// `partial`: also write the ||dF||^2 / ||dY||^2 partials (iterations that end in a control launch).
// `e0`, `e1` (may be null): events recorded by the dispatch itself at the start and the end of
// the kernel (for the roofline timing).
template <typename T>
hipError_t launch_edge(const Consts &c, const Bufs<T> &b, const PartLayout &pl, EdgeShape sh, bool check,
                       bool partial, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
template <typename T>
hipError_t launch_node(const Consts &c, const Bufs<T> &b, const PartLayout &pl, bool check, bool partial,
                       hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
template <typename T>
hipError_t launch_fused(const Consts &c, const Bufs<T> &b, const PartLayout &pl, EdgeShape sh, int parity,
                        bool check, bool partial, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
template <typename T>
hipError_t launch_residual(const Consts &c, const Bufs<T> &b, const PartLayout &pl, EdgeShape sh,
                           hipStream_t st);
// `adapt`: apply (e-primal_weight) if the step norms exceed tau; `k_inc`: iterations since the
// previous control launch (the device count advances by it).
template <typename T>
hipError_t launch_control(const Consts &c, const Bufs<T> &b, const PartLayout &pl, bool check, bool adapt,
                          long long k_inc, hipStream_t st);
template <typename T>
hipError_t launch_poison(const Bufs<T> &b, int which, long long offset, hipStream_t st);
// Two-phase iteration: P = F A^T recomputed from the current F (after F is set from outside).
template <typename T>
hipError_t launch_p_from_f(const Consts &c, const Bufs<T> &b, hipStream_t st);

int node_block_for(int n, int bytes);

// One slot of a batching pool: the instance and the values recorded when it was admitted.
// At pool iteration G the slot performs its iteration k = k0 + (G - G0), reading buffer set
// par0 ^ ((G - G0) & 1), until its stop flag is raised or k reaches max_iter.
template <typename T>
struct SlotDesc {
    Consts c;
    Bufs<T> b;
    PartLayout pl;
    long long G0, k0, max_iter;
    int par0, active;
};

// Device-resident state of a pool: its iteration counter and the sizes of its work lists.  The
// kernels of a step read G (iteration `it` of the step is G + it) and the list sizes from here,
// so a step's launches carry no value that changes between steps and can be replayed from a
// captured graph; the last launch of each step advances G.
struct PoolState {
    long long G;
    int nwork;  // fused node items (slot, node) of the batched iteration
    int nres;   // residual items (slot, block of RES_EDGES edges)
    int nedge;  // flat edge items of the two-phase slots (slot, block of EDGE_PAR_WAVES edges)
    int nnode;  // node items of the two-phase slots (slot, node j * ceil(n/64) + row block)
};

// Waves (one node item each) per workgroup of the pool's two-phase node launch.
constexpr int POOL_NODE_WAVES = 4;

// Launch shape of a pool: waves per node workgroup (1, 2, 4 or 8), the grids of the iteration and
// residual launches (the item counts rounded up; set per step), and the largest entries per lane
// of an admitted instance (1, 2, 4 or 8: n <= 64 ept).
struct PoolShape {
    int waves, grid, res_grid, max_ept;
    int edge_grid, node_grid;  // grids of the two-phase slots' edge and node launches (0: none)
};

template <typename T>
hipError_t launch_pool_iteration(const SlotDesc<T> *slots, const int2 *work, const int2 *ework, const int2 *nwork,
                                 const int *res_off, const PoolState *ps, int nslots, PoolShape sh, int it, bool check,
                                 bool control, hipStream_t st);
template <typename T>
hipError_t launch_pool_gather(const SlotDesc<T> *slots, int nslots, DevScalars *out, PoolState *ps, int iters,
                              hipStream_t st);
// the pool shapes compiled into the library, and the measured choice for a pool of iterate
// size `bytes` whose instances have at most n_max nodes
bool pool_waves_valid(int waves, int bytes);
PoolShape pool_shape_for(int n_max, int bytes);
// the organisation measured fastest in a saturated pool for an instance of n nodes: 0 = fused,
// 1 = two-phase (flat edge phase, 64-thread node blocks)
int pool_org_for(int n, int bytes);

}  // namespace mcf

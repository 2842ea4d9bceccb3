// libmcf device kernels for gfx950 (CDNA4, wave64).
//
// One PDHG iteration of Algorithm 2.1 (eq. (e-pdhg-step)) is two launches:
//   edge phase : per tail node t, for each edge column l leaving t (destination-major,
//                contiguous n-vector): q = F[:,l] + alpha (Y[:,head] - Y[:,tail]);
//                Fhat = (q - mu)_+ (the projection of Section 2.3, mu from an exact
//                active-set search); F <- rho Fhat + (1 - rho) F; the new columns of
//                the edges leaving t are summed into Sout[:,t].
//   node phase : per node column j: P' = F A^T of the new F, from a gather over the
//                in-edge list minus Sout[:,j].  Since Fbar = 2 Fhat - F_old and
//                F_new = rho Fhat + (1 - rho) F_old, Fbar = (2/rho) F_new - ((2-rho)/rho) F_old,
//                so V = Fbar A^T = (2/rho) P' - ((2-rho)/rho) P with P = F_old A^T kept from
//                the previous iteration: Fbar is never stored.  Yhat = prox(Y - beta V) off
//                the diagonal, 0 on it (Section 2.3); Y <- rho Yhat + (1 - rho) Y; P <- P'.
// Iterations that adapt the primal weight (k a multiple of k_adapt) or check the
// residual also write FP64 partials of ||dF||^2 and ||dY||^2 and end in a control
// launch: FP64 fixed-order reduction, (e-primal_weight), the stop flag.  On check
// iterations the edge and node phases also produce Fhat, D = Fhat - Q, T = -Fhat A^T
// and U' = u'(T), and a residual pass forms ||G||^2 and <G, D> for r(Q) of (e-res).
// No atomics anywhere: every sum has a fixed order, so results are deterministic.
#include <hip/hip_ext.h>
#include <math.h>

#include "mcf_internal.h"

namespace mcf {

// ------------------------------------------------------------------ reductions
// Wave-wide sums through DPP lane moves (quad xor 1, quad xor 2, row rotate 4 and 8)
// leave every lane of a 16-lane row with the row total; the four row totals, read
// from lanes 0/16/32/48, are added in row order.  The result is uniform (scalar) and
// its rounding order is fixed.
// The lane moves used here (quad permutes, row rotates) read a valid lane for every lane, so
// the destination's previous value is never kept and needs no initialisation.
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v)
{
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i32<CTRL>((int)(b & 0xffffffffLL));
    const int hi = dpp_i32<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double lane_f64(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

constexpr int DPP_QUAD_XOR1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int DPP_ROW_ROR4 = 0x124;
constexpr int DPP_ROW_ROR8 = 0x128;

__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_f64<DPP_QUAD_XOR1>(v);
    v += dpp_f64<DPP_QUAD_XOR2>(v);
    v += dpp_f64<DPP_ROW_ROR4>(v);
    v += dpp_f64<DPP_ROW_ROR8>(v);
    return ((lane_f64(v, 0) + lane_f64(v, 16)) + lane_f64(v, 32)) + lane_f64(v, 48);
}

// Two wave sums with their DPP steps interleaved, so that the two dependency chains overlap;
// each result is bitwise the one wave_sum gives.
__device__ __forceinline__ void wave_sum2(double &x, double &y)
{
    x += dpp_f64<DPP_QUAD_XOR1>(x);
    y += dpp_f64<DPP_QUAD_XOR1>(y);
    x += dpp_f64<DPP_QUAD_XOR2>(x);
    y += dpp_f64<DPP_QUAD_XOR2>(y);
    x += dpp_f64<DPP_ROW_ROR4>(x);
    y += dpp_f64<DPP_ROW_ROR4>(y);
    x += dpp_f64<DPP_ROW_ROR8>(x);
    y += dpp_f64<DPP_ROW_ROR8>(y);
    x = ((lane_f64(x, 0) + lane_f64(x, 16)) + lane_f64(x, 32)) + lane_f64(x, 48);
    y = ((lane_f64(y, 0) + lane_f64(y, 16)) + lane_f64(y, 32)) + lane_f64(y, 48);
}

// 1/k from the per-instance table (k = 1..n), read through the constant address space with a
// wave-uniform k: a scalar load.  A vector load here would make the search wait for every
// vector memory operation still in flight (the next edge's column loads, the stores just
// issued), since those waits count all of them.
__device__ __forceinline__ double rcp_of(const double *tab, int k)
{
    typedef const __attribute__((address_space(4))) double cdouble;
    return ((cdouble *)tab)[__builtin_amdgcn_readfirstlane(k)];
}

// Number of lanes of the wave for which p holds (wave-uniform): a ballot, no reduction chain.
__device__ __forceinline__ int wave_count(bool p)
{
    return __popcll(__ballot(p));
}

__device__ __forceinline__ int wave_sum(int v)
{
    v += dpp_i32<DPP_QUAD_XOR1>(v);
    v += dpp_i32<DPP_QUAD_XOR2>(v);
    v += dpp_i32<DPP_ROW_ROR4>(v);
    v += dpp_i32<DPP_ROW_ROR8>(v);
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
           __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}

__device__ __forceinline__ double wave_max(double v)
{
    v = fmax(v, dpp_f64<DPP_QUAD_XOR1>(v));
    v = fmax(v, dpp_f64<DPP_QUAD_XOR2>(v));
    v = fmax(v, dpp_f64<DPP_ROW_ROR4>(v));
    v = fmax(v, dpp_f64<DPP_ROW_ROR8>(v));
    return fmax(fmax(lane_f64(v, 0), lane_f64(v, 16)), fmax(lane_f64(v, 32), lane_f64(v, 48)));
}

// Sums over a group of NW waves (one edge column or one node block): wave sums,
// then the NW wave totals added in wave order through LDS.  NW == 1 needs no LDS.
// `lds` must hold 2*NW doubles and be private to the group.
template <int NW>
__device__ __forceinline__ void group_sum(double &x, double &y, double *lds)
{
    x = wave_sum(x);
    y = wave_sum(y);
    if constexpr (NW > 1) {
        const int lane = threadIdx.x & 63, wid = (threadIdx.x >> 6) % NW;
        __syncthreads();
        if (lane == 0) {
            lds[wid] = x;
            lds[NW + wid] = y;
        }
        __syncthreads();
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            sx += lds[w];
            sy += lds[NW + w];
        }
        x = sx;
        y = sy;
    }
}

template <int NW>
__device__ __forceinline__ void group_sum(double &x, int &y, double *lds)
{
    x = wave_sum(x);
    y = wave_sum(y);
    if constexpr (NW > 1) {
        const int lane = threadIdx.x & 63, wid = (threadIdx.x >> 6) % NW;
        __syncthreads();
        if (lane == 0) {
            lds[wid] = x;
            lds[NW + wid] = (double)y;
        }
        __syncthreads();
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            sx += lds[w];
            sy += lds[NW + w];
        }
        x = sx;
        y = (int)sy;
    }
}

// Adds K wave-uniform values over the NW waves of a group, in wave order, through LDS
// (`lds` holds K * NW doubles and is private to the group).  NW == 1 needs nothing.
template <int NW, int K>
__device__ __forceinline__ void group_combine(double (&x)[K], double *lds)
{
    if constexpr (NW > 1) {
        const int lane = threadIdx.x & 63, wid = (threadIdx.x >> 6) % NW;
        __syncthreads();
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) lds[k * NW + wid] = x[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) s += lds[k * NW + w];
            x[k] = s;
        }
    }
}

template <int NW>
__device__ __forceinline__ double group_max(double x, double *lds)
{
    x = wave_max(x);
    if constexpr (NW > 1) {
        const int lane = threadIdx.x & 63, wid = (threadIdx.x >> 6) % NW;
        __syncthreads();
        if (lane == 0) lds[wid] = x;
        __syncthreads();
        double m = -INFINITY;
#pragma unroll
        for (int w = 0; w < NW; ++w) m = fmax(m, lds[w]);
        x = m;
    }
    return x;
}

// --------------------------------------------------------------- utilities
// Section 1.1: u(s) = w log s (UTIL 0), w s^g (UTIL 1, power, g = gamma) or the alpha-fair
// w s^{1-g} / (1-g) (UTIL 2, g = alpha); u' for U' = u'(T); the traffic s(y) maximizing
// y s + u(s), from u'(s) = -y, and the conjugate (-u)^*(y) = y s(y) + u(s(y)), both for y < 0.
// For the alpha-fair utility w s^{1-g} = -y s at s = s(y), so the conjugate is (-y) s g/(1-g).
// UTIL 3 is the power utility with g = 1/2 known when compiling: the same operations as UTIL 1
// at g = 1/2, without the code of the general exponent (which sets the register count of the
// node launch).
constexpr int UTIL_POWER_HALF = 3;
template <int UTIL>
__device__ __forceinline__ double util_u(double s, double w, double g)
{
    if (UTIL == 0) return w * log(s);
    if (UTIL == 1 || UTIL == UTIL_POWER_HALF) return w * pow(s, g);
    return w * pow(s, 1.0 - g) / (1.0 - g);
}
template <int UTIL>
__device__ __forceinline__ double util_du(double s, double w, double g)
{
    if (UTIL == 0) return w / s;
    if (UTIL == 1 || UTIL == UTIL_POWER_HALF) return w * g * pow(s, g - 1.0);
    return w * pow(s, -g);
}
template <int UTIL>
__device__ __forceinline__ double util_traffic(double y, double w, double g)
{
    if (UTIL == 0) return w / (-y);
    if (UTIL == 1 || UTIL == UTIL_POWER_HALF) return pow(w * g / (-y), 1.0 / (1.0 - g));
    return pow(w / (-y), 1.0 / g);
}
template <int UTIL>
__device__ __forceinline__ double util_conj(double y, double w, double g)
{
    if (UTIL == 0) return -w + w * log(w) - w * log(-y);
    if (UTIL == 1 || UTIL == UTIL_POWER_HALF)
        return (1.0 / g - 1.0) * pow(w * g, 1.0 / (1.0 - g)) * pow(-y, -g / (1.0 - g));
    return (-y) * util_traffic<2>(y, w, g) * g / (1.0 - g);
}

// Dual proximal operator prox_{beta (-u)^*}(y) of Section 2.3.
//   log:   (y - sqrt(y^2 + 4 beta w)) / 2, in the cancellation-free form for y > 0;
//   power: z = -t with t the positive root of h(t) = t^{c1+2} + y t^{c1+1} - c1 c2.  On
//          t >= a = max(-y, 0) h is increasing and convex, so Newton's method decreases
//          monotonically onto the root from any point right of it, and one step from a
//          point left of it (in [a, root)) lands right of it.  The start is the guess
//          `tg` (the current dual value, -Y_ij, which the new root is close to once the
//          iteration settles) when it lies in the bracket [a, a + (c1 c2)^{1/(c1+2)}], else
//          the bracket's right end; iteration stops when a step no longer decreases t.
//   alpha-fair: the optimality condition z + beta s(z) = y gives, with t = -z and p = 1/alpha
//          (passed as c1), h(t) = t^p (t + y) - beta w^p = 0 on the same kind of bracket.  For
//          alpha > 1 (p < 1) and y > 0, h is concave near 0, where a Newton step from the right
//          can leave the bracket; so the bracket [lo, hi] is kept by the sign of h and a step
//          that leaves it is replaced by bisection (safeguarded Newton).
template <int UTIL>
__device__ __forceinline__ double prox_alpha(double y, double beta, double w, double p, double tg)
{
    const double a = y < 0.0 ? -y : 0.0;
    const double k = beta * pow(w, p);
    double lo = a, hi = a + pow(k, 1.0 / (p + 1.0));  // h(lo) < 0 <= h(hi)
    double t = (tg > lo && tg < hi) ? tg : hi;
    for (int it = 0; it < 200; ++it) {
        const double tq = pow(t, p - 1.0);
        const double h = tq * t * (t + y) - k;
        if (h == 0.0) break;
        if (h < 0.0) lo = t;
        else hi = t;
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;  // the bracket is two adjacent doubles
        double tn = t - h / (tq * fma(p + 1.0, t, p * y));
        if (!(tn > lo && tn < hi)) tn = mid;
        if (tn == t) break;
        t = tn;
    }
    return -t;
}

// A sum of two products is written as one explicit fma: left to the compiler, which product
// it fuses can depend on the code around the call, and so the rounding could differ between
// kernels that share this code.
template <int UTIL>
__device__ __forceinline__ double prox_dual(double y, double beta, double w, double g, double c1, double tg)
{
    if (UTIL == 0) {
        const double s = sqrt(fma(y, y, 4.0 * beta * w));
        return y <= 0.0 ? 0.5 * (y - s) : -2.0 * beta * w / (y + s);
    }
    if (UTIL == 2) return prox_alpha<UTIL>(y, beta, w, c1, tg);
    const double a = y < 0.0 ? -y : 0.0;
    const bool half = UTIL == UTIL_POWER_HALF || c1 == 1.0;  // gamma = 1/2: t^3 + y t^2 - beta w^2 / 4
    const double k = half ? beta * w * w * 0.25 : c1 * beta * (1.0 / g - 1.0) * pow(w * g, 1.0 / (1.0 - g));
    auto hval = [&](double t, double &hp) {
        const double tp = half ? t : pow(t, c1);
        hp = tp * fma(c1 + 2.0, t, (c1 + 1.0) * y);
        return tp * t * (t + y) - k;
    };
    const double hi = a + (half ? cbrt(k) : pow(k, 1.0 / (c1 + 2.0)));
    double t = (tg > a && tg < hi) ? tg : hi;
    double hp;
    const double h0 = hval(t, hp);
    if (h0 < 0.0) t = t - h0 / hp;  // from left of the root: one step lands right of it
    for (int it = 0; it < 200; ++it) {
        const double h = hval(t, hp);
        const double tn = t - h / hp;
        if (!(tn < t)) break;
        t = tn > a ? tn : a;
    }
    return -t;
}

// ------------------------------------------------------------- XCD mapping
// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).  Mapping launch
// index b to work item (b % 8) * per + b / 8 gives every XCD one contiguous range of work
// items, so neighbours in the work order (edges with the same tail) share an L2.  The grid
// has 8 * per workgroups; those mapped past `items` return at once.
constexpr int NUM_XCD = 8;

__device__ __forceinline__ int xcd_item(int b, int items)
{
    const int per = (items + NUM_XCD - 1) / NUM_XCD;
    return (b % NUM_XCD) * per + b / NUM_XCD;
}

inline int xcd_grid(int items) { return ((items + NUM_XCD - 1) / NUM_XCD) * NUM_XCD; }

// ------------------------------------------------------------------- init
template <typename T>
__global__ void init_kernel(Consts c, Bufs<T> b, double omega0)
{
    const long long nm = c.ld * (long long)c.m, nn = c.ld * (long long)c.n;
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (long long x = t0; x < nm; x += stride) {
        b.F[x] = T(0);
        b.Fhat[x] = T(0);
    }
    for (long long x = t0; x < nn; x += stride) {
        const long long j = x / c.ld, i = x - j * c.ld;
        // Section 2.5 initialization: Y^0 = I - 1 1^T (0 on the diagonal, -1 off it); padding stays 0.
        b.Y[x] = (i < c.n && i != j) ? T(-1) : T(0);
        b.That[x] = 0.0;
        if (!c.fused) b.P[x] = T(0);  // P = F A^T of F = 0
    }
    for (long long x = t0; x < c.m; x += stride) b.mu[x] = 0.0;
    if (t0 == 0) {
        DevScalars *sc = b.sc;
        sc->omega = omega0;
        sc->alpha = sc->eta / omega0;
        sc->beta = sc->eta * omega0;
        sc->dF = sc->dY = 0.0;
        sc->r = sc->r_paper = sc->rel_primal = sc->rel_dual = sc->rel_gap = sc->rel_kkt = INFINITY;
        sc->primal_obj = INFINITY;
        sc->dual_obj = -INFINITY;
        sc->infeasible_frac = 1.0;
        sc->a = sc->b = sc->e = 0.0;
        sc->k = 0;
        sc->stop = 0;
        sc->state = 0;
        sc->checked = 0;
    }
}

// -------------------------------------------------------------- edge phase
// 16-byte vectors of the iterate type: 4 floats or 2 doubles.
template <typename T> struct Vec;
template <> struct Vec<float> { using type = float4; static constexpr int N = 4; };
template <> struct Vec<double> { using type = double2; static constexpr int N = 2; };

template <typename T>
__device__ __forceinline__ void vload(const T *p, T (&x)[Vec<T>::N])
{
    const typename Vec<T>::type v = *reinterpret_cast<const typename Vec<T>::type *>(p);
    if constexpr (Vec<T>::N == 4) { x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w; }
    else { x[0] = v.x; x[1] = v.y; }
}

template <typename T>
__device__ __forceinline__ void vstore(T *p, const T (&x)[Vec<T>::N])
{
    typename Vec<T>::type v;
    if constexpr (Vec<T>::N == 4) { v.x = x[0]; v.y = x[1]; v.z = x[2]; v.w = x[3]; }
    else { v.x = x[0]; v.y = x[1]; }
    *reinterpret_cast<typename Vec<T>::type *>(p) = v;
}

// Streaming (non-temporal) forms for data touched once per iteration, so that the lines that
// are reused (a tail's Y column, read once per out-edge) keep their place in the L2.
template <typename T> struct NtVec;
template <> struct NtVec<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct NtVec<double> { typedef double type __attribute__((ext_vector_type(2))); };

template <typename T>
__device__ __forceinline__ void vload_nt(const T *p, T (&x)[Vec<T>::N])
{
    const typename NtVec<T>::type v = __builtin_nontemporal_load(reinterpret_cast<const typename NtVec<T>::type *>(p));
#pragma unroll
    for (int u = 0; u < Vec<T>::N; ++u) x[u] = v[u];
}

template <typename T>
__device__ __forceinline__ void vstore_nt(T *p, const T (&x)[Vec<T>::N])
{
    typename NtVec<T>::type v;
#pragma unroll
    for (int u = 0; u < Vec<T>::N; ++u) v[u] = x[u];
    __builtin_nontemporal_store(v, reinterpret_cast<typename NtVec<T>::type *>(p));
}

// The largest value of type T that is <= x: for q of type T, q > x exactly when q > below(x).
__device__ __forceinline__ float below(double x, float) { return __double2float_rd(x); }
__device__ __forceinline__ double below(double x, double) { return x; }

// WPE waves per tail node t (WPE == 1: a 256-thread block carries 4 tail nodes, one per
// wave); they project the edges leaving t one after another, each lane holding NV 16-byte
// vectors of F[:,l] and q.  Vector v of lane x covers entries (v * 64 * WPE + x) * VEC ..
// + VEC - 1; a vector that starts below n is loaded whole: the padding rows n .. ld-1 of F
// and Y are zero, so their q is 0 and they never enter a support.
// mu (Section 2.3, Section 2.6): mu = 0 if sum (q)_+ <= c; otherwise the support S and
// mu = (sum_S q - c)/|S| satisfy S = {q > mu}.  Any mu' with S' = {q > mu'} nonempty
// gives the lower bound (sum_{S'} q - c)/|S'| <= mu (the linear function it zeroes lies
// below the convex piecewise-linear sum (q - x)_+ - c); from a lower bound the
// active-set iteration S <- {q > mu}, mu <- (sum_S q - c)/|S| rises monotonically and
// stops exactly when |S| stops shrinking.  The search starts from the larger of the
// bounds given by S' = {q > 0} and S' = {q > mu of the previous iteration}, so a
// column whose support did not move needs two block sums instead of five or six.
// The new columns of the edges leaving t are added, in edge order and in the iterate type,
// into Sout[:,t], the out-edge half of P' = F A^T.  (In FP32 that sum of the few columns
// leaving a node carries rounding of the same order as the FP32 columns themselves.)
// The partial and check variants of the 8-wave shapes whose regular variant fits 4 waves per SIMD
// (up to 6 vectors per lane) are held to 128 VGPRs too, so that they also keep 2 workgroups per CU:
// left alone the FP32 6-vector ones take 130 and 146 and fit one.  Held, the partial one spills 1
// register and runs 2.30 ms instead of 3.20 at n = 1e4, and the check one spills 19 and runs
// 4.69 ms instead of 4.71.
template <typename T, int WPE, int NV, bool CHECK, bool PARTIAL>
__global__ __launch_bounds__(WPE == 1 ? 256 : 64 * WPE)
__attribute__((amdgpu_waves_per_eu(WPE == 8 && NV <= 6 && (CHECK || PARTIAL) ? 4 : 1))) void edge_kernel(Consts c, Bufs<T> b, PartLayout pl)
{
    constexpr int VEC = Vec<T>::N;
    constexpr int LANES = 64 * WPE;  // threads per tail node
    constexpr int NT = WPE == 1 ? 256 : 64 * WPE;
    __shared__ double lds[4 * WPE];
    // the out-edge sums live in LDS, one 16-byte vector per (vector slot, thread): in
    // registers they would cost the occupancy that keeps enough loads in flight
    __shared__ typename Vec<T>::type sol[NV * NT];
    if (b.sc->stop) return;
    const int items = WPE == 1 ? (c.n + 3) / 4 : c.n;
    const int blk = xcd_item(blockIdx.x, items);
    if (blk >= items) return;
    const int tn = WPE == 1 ? blk * 4 + (int)(threadIdx.x >> 6) : blk;
    if (tn >= c.n) return;  // whole waves only (WPE == 1): no block barrier follows
    const int t = WPE == 1 ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
    const int n = c.n;
    const long long ld = c.ld;
    const T ta = (T)b.sc->alpha;
    const T *yt = b.Y + (long long)tn * ld;
    const double rho = c.rho, omr = 1.0 - c.rho;
    typename Vec<T>::type *so = sol + threadIdx.x;  // slot v at so[v * NT]
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const T z[VEC] = {};
        vstore(reinterpret_cast<T *>(so + v * NT), z);
    }
    const int e0 = b.out_off[tn], e1 = b.out_off[tn + 1];
    double dF_t = 0.0, e_t = 0.0, sup_t = 0.0;  // this tail's partials, edge by edge in order
    for (int e = e0; e < e1; ++e) {
        // e is uniform within the wave, so is its head: keep the column address scalar
        const T *yh = b.Y + (long long)__builtin_amdgcn_readfirstlane(b.head[e]) * ld;
        T *f = b.F + (long long)e * ld;
        const double cap = b.cap[e];
        const double mu0 = b.mu[e];
        // All 3 NV loads are issued before any is used: a vector past n reads the column's
        // first vector instead (always in bounds) and is then replaced by zeros.  F streams
        // (non-temporal loads and stores: each column is touched once per phase); Y[:,head]
        // takes ordinary loads, since each column of Y is read again at every edge that ends
        // there and the caches can serve some of those reads.
        T fo[NV][VEC], q[NV][VEC], bh[NV][VEC], bt[NV][VEC];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int i = (v * LANES + t) * VEC;
            const int ic = i < n ? i : 0;
            vload_nt(f + ic, fo[v]);
            vload(yh + ic, bh[v]);
            vload(yt + ic, bt[v]);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const bool ok = (v * LANES + t) * VEC < n;
#pragma unroll
            for (int u = 0; u < VEC; ++u) {
                q[v][u] = ok ? fo[v][u] + ta * (bh[v][u] - bt[v][u]) : T(0);
                fo[v][u] = ok ? fo[v][u] : T(0);
            }
        }
        // Sums over a support {q > thr}: each 16-byte vector is first added in the iterate
        // type (in a fixed order), then in FP64.  Converting per vector rather than per entry
        // keeps the compiler from holding an FP64 copy of every q across the passes.
        // The support sizes are counted wave by wave with ballots (no reduction chain).
        auto support_sum = [&](T thr, double &s, int &cnt) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                T part = T(0);
#pragma unroll
                for (int u = 0; u < VEC; ++u) {
                    const bool in = q[v][u] > thr;
                    if (in) part += q[v][u];
                    cnt += wave_count(in);
                }
                s += (double)part;
            }
        };
        const T thr0 = below(mu0, T(0));
        double sp = 0.0, sw = 0.0;
        int cp = 0, cw = 0;
        support_sum(T(0), sp, cp);
        support_sum(thr0, sw, cw);
        wave_sum2(sp, sw);
        {
            double g[4] = {sp, sw, (double)cp, (double)cw};
            group_combine<WPE, 4>(g, lds);
            sp = g[0];
            sw = g[1];
            cp = (int)g[2];
            cw = (int)g[3];
        }
        double mu = 0.0;
        if (sp > cap) {
            mu = (sp - cap) * rcp_of(b.rcp, cp);
            int prev = cp;  // mu came from S' = {q > 0}, a superset of {q > mu}
            if (cw > 0) {
                const double mw = (sw - cap) * rcp_of(b.rcp, cw);
                if (mw > mu) {
                    mu = mw;
                    prev = mw >= mu0 ? cw : 0x7fffffff;  // {q > mu0} contains {q > mw} only if mw >= mu0
                }
            }
            // each pass counts the support first; only a support that shrank needs its sum
            for (int pass = 0; pass <= n; ++pass) {
                const T thr = below(mu, T(0));
                int cnt = 0;
#pragma unroll
                for (int v = 0; v < NV; ++v)
#pragma unroll
                    for (int u = 0; u < VEC; ++u) cnt += wave_count(q[v][u] > thr);
                {
                    double g[1] = {(double)cnt};
                    group_combine<WPE, 1>(g, lds);
                    cnt = (int)g[0];
                }
                if (cnt >= prev) break;
                double s = 0.0;
                int dummy = 0;
                support_sum(thr, s, dummy);
                s = wave_sum(s);
                {
                    double g[1] = {s};
                    group_combine<WPE, 1>(g, lds);
                    s = g[0];
                }
                mu = (s - cap) * rcp_of(b.rcp, cnt);
                prev = cnt;
            }
        }
        double dsum = 0.0, esum = 0.0, gmax = -INFINITY;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int i = (v * LANES + t) * VEC;
            if (i < n) {
                T fn[VEC], fhv[VEC], dv[VEC], sv[VEC];
                vload(reinterpret_cast<const T *>(so + v * NT), sv);
#pragma unroll
                for (int u = 0; u < VEC; ++u) {
                    // widen F here, not at its load: an FP64 copy of every entry held across
                    // the multiplier search would double the registers the column takes
                    T fov = fo[v][u];
                    asm volatile("" : "+v"(fov));
                    const double fod = (double)fov;
                    const double fh = fmax((double)q[v][u] - mu, 0.0);
                    fn[u] = (T)(rho * fh + omr * fod);
                    sv[u] += fn[u];
                    if (PARTIAL) {
                        const double d = (double)fn[u] - fod;
                        dsum += d * d;
                    }
                    if (CHECK) {
                        fhv[u] = (T)fh;
                        dv[u] = (T)(fh - (double)q[v][u]);
                        esum += (double)dv[u] * (double)dv[u];
                    }
                }
                vstore_nt(f + i, fn);
                vstore(reinterpret_cast<T *>(so + v * NT), sv);
                if (CHECK) {
                    vstore_nt(b.Fhat + (long long)e * ld + i, fhv);
                    vstore_nt(b.D + (long long)e * ld + i, dv);
                    T bh[VEC], bt[VEC];
                    vload(yh + i, bh);
                    vload(yt + i, bt);
#pragma unroll
                    for (int u = 0; u < VEC; ++u)
                        if (i + u < n) gmax = fmax(gmax, (double)(bh[u] - bt[u]));
                }
            }
        }
        if (PARTIAL) group_sum<WPE>(dsum, esum, lds);
        if (CHECK) gmax = group_max<WPE>(gmax, lds);
        if (t == 0) b.mu[e] = mu;
        dF_t += dsum;
        e_t += esum;
        if (CHECK) sup_t += cap * fmax(gmax, 0.0);  // c_l (max_i (Y A)_il)_+
    }
    if (t == 0) {
        if (PARTIAL) b.part[pl.dF + tn] = dF_t;
        if (CHECK) {
            b.part[pl.e + tn] = e_t;
            b.part[pl.sup + tn] = sup_t;
        }
    }
    T *sout = b.Sout + (long long)tn * ld;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int i = (v * LANES + t) * VEC;
        if (i < n) {  // non-temporal: the node phase reads Sout once, and Y keeps the caches
            T sv[VEC];
            vload(reinterpret_cast<const T *>(so + v * NT), sv);
            vstore_nt(sout + i, sv);
        }
    }
}

// One edge column projected by one wave (n <= 64 * NV * VEC), with wave-level reductions only:
// q = F[:,e] + alpha (Y[:,head] - Y[:,tail]), the multiplier mu by the warm-started active-set
// search of edge_kernel, F <- rho Fhat + (1 - rho) F.  With OUTSUM the new column is added (in
// the iterate type) into this lane's slice `so` of the wave's out-edge sum in LDS.  Adds the
// edge's ||dF||^2, ||D||^2 and support term c_l (max_i (Y A)_il)_+ to the wave's totals.
template <typename T, int NV, bool CHECK, bool PARTIAL, bool OUTSUM>
__device__ __forceinline__ void wave_edge(const Consts &c, const Bufs<T> &b, int e, const T *yt, T ta, T *so,
                                          double &dF_w, double &e_w, double &sup_w)
{
    constexpr int VEC = Vec<T>::N;
    const int t = threadIdx.x & 63;
    const int n = c.n;
    const long long ld = c.ld;
    const double rho = c.rho, omr = 1.0 - c.rho;
    const T *yh = b.Y + (long long)__builtin_amdgcn_readfirstlane(b.head[e]) * ld;
    T *f = b.F + (long long)e * ld;
    const double cap = b.cap[e];
    const double mu0 = b.mu[e];
    T fo[NV][VEC], q[NV][VEC], bh[NV][VEC], bt[NV][VEC];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int i = (v * 64 + t) * VEC;
        const int ic = i < n ? i : 0;
        if (c.f_cached) vload(f + ic, fo[v]);  // see F_CACHED_BYTES
        else vload_nt(f + ic, fo[v]);
        vload(yh + ic, bh[v]);
        vload(yt + ic, bt[v]);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const bool ok = (v * 64 + t) * VEC < n;
#pragma unroll
        for (int u = 0; u < VEC; ++u) {
            q[v][u] = ok ? fo[v][u] + ta * (bh[v][u] - bt[v][u]) : T(0);
            fo[v][u] = ok ? fo[v][u] : T(0);
        }
    }
    auto support_sum = [&](T thr, double &s, int &cnt) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T part = T(0);
#pragma unroll
            for (int u = 0; u < VEC; ++u) {
                const bool in = q[v][u] > thr;
                if (in) part += q[v][u];
                cnt += wave_count(in);
            }
            s += (double)part;
        }
    };
    const T thr0 = below(mu0, T(0));
    double sp = 0.0, sw = 0.0;
    int cp = 0, cw = 0;
    support_sum(T(0), sp, cp);
    support_sum(thr0, sw, cw);
    wave_sum2(sp, sw);
    double mu = 0.0;
    if (sp > cap) {
        mu = (sp - cap) * rcp_of(b.rcp, cp);
        int prev = cp;  // mu came from S' = {q > 0}, a superset of {q > mu}
        if (cw > 0) {
            const double mw = (sw - cap) * rcp_of(b.rcp, cw);
            if (mw > mu) {
                mu = mw;
                prev = mw >= mu0 ? cw : 0x7fffffff;  // {q > mu0} contains {q > mw} only if mw >= mu0
            }
        }
        // each pass counts the support first; only a support that shrank needs its sum
        for (int pass = 0; pass <= n; ++pass) {
            const T thr = below(mu, T(0));
            int cnt = 0;
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int u = 0; u < VEC; ++u) cnt += wave_count(q[v][u] > thr);
            if (cnt >= prev) break;
            double s = 0.0;
            int dummy = 0;
            support_sum(thr, s, dummy);
            s = wave_sum(s);
            mu = (s - cap) * rcp_of(b.rcp, cnt);
            prev = cnt;
        }
    }
    double dsum = 0.0, esum = 0.0, gmax = -INFINITY;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int i = (v * 64 + t) * VEC;
        if (i < n) {
            T fn[VEC], fhv[VEC], dv[VEC], acc[VEC];
            if (OUTSUM) vload(so + v * 64 * VEC, acc);
#pragma unroll
            for (int u = 0; u < VEC; ++u) {
                T fov = fo[v][u];
                asm volatile("" : "+v"(fov));
                const double fod = (double)fov;
                const double fh = fmax((double)q[v][u] - mu, 0.0);
                fn[u] = (T)(rho * fh + omr * fod);
                if (OUTSUM) acc[u] += fn[u];
                if (PARTIAL) {
                    const double d = (double)fn[u] - fod;
                    dsum += d * d;
                }
                if (CHECK) {
                    fhv[u] = (T)fh;
                    dv[u] = (T)(fh - (double)q[v][u]);
                    esum += (double)dv[u] * (double)dv[u];
                }
            }
            if (OUTSUM) vstore(so + v * 64 * VEC, acc);
            if (c.f_cached) vstore(f + i, fn);
            else vstore_nt(f + i, fn);
            if (CHECK) {
                vstore_nt(b.Fhat + (long long)e * ld + i, fhv);
                vstore_nt(b.D + (long long)e * ld + i, dv);
#pragma unroll
                for (int u = 0; u < VEC; ++u)
                    if (i + u < n) gmax = fmax(gmax, (double)(bh[v][u] - bt[v][u]));
            }
        }
    }
    if (PARTIAL) dsum = wave_sum(dsum);
    if (CHECK) {
        esum = wave_sum(esum);
        gmax = wave_max(gmax);
    }
    if (t == 0) b.mu[e] = mu;
    dF_w += dsum;
    e_w += esum;
    if (CHECK) sup_w += cap * fmax(gmax, 0.0);  // c_l (max_i (Y A)_il)_+
}

// Concurrent edge phase for columns that fit one wave (n <= 64 * NV * VEC): workgroup =
// tail node t with EDGE_PAR_WAVES waves; wave w projects the out-edges e0 + w, e0 + w + NW, ...
// with wave-level reductions only (wave_edge), so the waves never wait for each other inside
// the loop.  Each wave adds its new columns into its own out-sum (in the iterate type, in its
// edge order); the sums are then added over the waves in wave order through LDS into
// Sout[:,t].  Partials per tail: wave totals added in wave order.
template <typename T, int NV, bool CHECK, bool PARTIAL>
__global__ __launch_bounds__(64 * EDGE_PAR_WAVES) __attribute__((amdgpu_waves_per_eu(NV == 4 && !CHECK ? 6 : 1)))
void edge_kernel_par(Consts c, Bufs<T> b, PartLayout pl)
{
    constexpr int VEC = Vec<T>::N;
    constexpr int NW = EDGE_PAR_WAVES;
    constexpr int COL = 64 * NV * VEC;  // entries of one column held by a wave
    __shared__ __attribute__((aligned(16))) T sol[NW * COL];
    __shared__ double red[3 * NW];
    if (b.sc->stop) return;
    const int tn = xcd_item(blockIdx.x, c.n);
    if (tn >= c.n) return;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), t = threadIdx.x & 63;
    const int n = c.n;
    const long long ld = c.ld;
    const T ta = (T)b.sc->alpha;
    const T *yt = b.Y + (long long)tn * ld;
    const int e0 = b.out_off[tn], e1 = b.out_off[tn + 1];
    // this wave's out-edge sum lives in its own slice of sol (registers are what limit how many
    // workgroups a CU holds; each lane touches only its own entries until the barrier)
    T *so = sol + w * COL + t * VEC;
    {
        T z[VEC];
#pragma unroll
        for (int u = 0; u < VEC; ++u) z[u] = T(0);
#pragma unroll
        for (int v = 0; v < NV; ++v) vstore(so + v * 64 * VEC, z);
    }
    double dF_w = 0.0, e_w = 0.0, sup_w = 0.0;
    for (int e = e0 + w; e < e1; e += NW) wave_edge<T, NV, CHECK, PARTIAL, true>(c, b, e, yt, ta, so, dF_w, e_w, sup_w);
    // out-edge sums over the waves, in wave order
    if (t == 0) {
        red[w] = dF_w;
        red[NW + w] = e_w;
        red[2 * NW + w] = sup_w;
    }
    __syncthreads();
    T *sout = b.Sout + (long long)tn * ld;
    for (int i = threadIdx.x; i < n; i += 64 * NW) {
        T acc = T(0);
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) acc += sol[ww * COL + i];
        sout[i] = acc;
    }
    if (threadIdx.x == 0) {
        double a = 0.0, bb = 0.0, cc = 0.0;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
            a += red[ww];
            bb += red[NW + ww];
            cc += red[2 * NW + ww];
        }
        if (PARTIAL) b.part[pl.dF + tn] = a;
        if (CHECK) {
            b.part[pl.e + tn] = bb;
            b.part[pl.sup + tn] = cc;
        }
    }
}

// Flat edge phase for columns that fit one wave: workgroup b = edges b NW .. b NW + NW - 1 (the
// internal order, sorted by tail, so the edges of a workgroup mostly share their tail column),
// one wave per edge, nothing shared between the waves: no projection waits for another edge,
// and no tail's out-edges form a second round.  The out-edge sums are left to the node phase,
// which gathers the out-edges of F as well as the in-edges.  Partials per workgroup: wave
// totals added in wave order.
// Workgroup `blk` of the flat edge phase (EDGE_PAR_WAVES waves, edges blk NW + wave); the wave
// totals of its partials are added in wave order through `red` (3 NW doubles).  Every wave of
// the workgroup calls it with the same blk.
template <typename T, int NV, bool CHECK, bool PARTIAL>
__device__ __forceinline__ void flat_block(const Consts &c, const Bufs<T> &b, const PartLayout &pl, int blk,
                                           double *red)
{
    constexpr int NW = EDGE_PAR_WAVES;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), t = threadIdx.x & 63;
    const int e = blk * NW + w;
    double dF_w = 0.0, e_w = 0.0, sup_w = 0.0;
    if (e < c.m) {
        const T *yt = b.Y + (long long)__builtin_amdgcn_readfirstlane(b.tail[e]) * c.ld;
        wave_edge<T, NV, CHECK, PARTIAL, false>(c, b, e, yt, (T)b.sc->alpha, nullptr, dF_w, e_w, sup_w);
    }
    if (!PARTIAL && !CHECK) return;
    if (t == 0) {
        red[w] = dF_w;
        red[NW + w] = e_w;
        red[2 * NW + w] = sup_w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, bb = 0.0, cc = 0.0;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
            a += red[ww];
            bb += red[NW + ww];
            cc += red[2 * NW + ww];
        }
        if (PARTIAL) b.part[pl.dF + blk] = a;
        if (CHECK) {
            b.part[pl.e + blk] = bb;
            b.part[pl.sup + blk] = cc;
        }
    }
}

template <typename T, int NV, bool CHECK, bool PARTIAL>
__global__ __launch_bounds__(64 * EDGE_PAR_WAVES) void edge_kernel_flat(Consts c, Bufs<T> b, PartLayout pl)
{
    __shared__ double red[3 * EDGE_PAR_WAVES];
    if (b.sc->stop) return;
    const int blk = xcd_item(blockIdx.x, c.nep);
    if (blk >= c.nep) return;
    flat_block<T, NV, CHECK, PARTIAL>(c, b, pl, blk, red);
}

// -------------------------------------------------------------- node phase
// Grid (ceil(n/NB), n): thread (x, j) owns entry i of node column j.  Gathers over the
// CSR edge lists accumulate in FP64 in list order.  Loads are issued sixteen edges at a time
// and unconditionally (a slot past the list end reloads an edge of the list and adds nothing),
// so a node with up to 16 edges in a list costs one round trip to memory.
// WIDE (the latency form): the sixteen edge ids of a batch are one scalar load (the in-edge
// list carries IN_EDGE_PAD entries past its end, so the load never leaves it) and all sixteen
// column loads are issued before the first add waits.  Otherwise each id is loaded on its own
// and the compiler interleaves the column loads with the adds, fewer of them in flight.
template <typename T, bool WIDE = false>
__device__ __forceinline__ double gather_in(const T *X, const int *in_edge, int i0, int i1, long long ld, int i)
{
    constexpr int B = 16;
    static_assert(B <= IN_EDGE_PAD, "a batch of edge ids may read past the list end");
    typedef const __attribute__((address_space(4))) int cint;
    double v = 0.0;
    for (int k = i0; k < i1; k += B) {
        T a[B];
        if (WIDE) {
            int id[B];
#pragma unroll
            for (int u = 0; u < B; ++u) id[u] = ((cint *)in_edge)[k + u];
#pragma unroll
            for (int u = 0; u < B; ++u) a[u] = X[(long long)(k + u < i1 ? id[u] : id[0]) * ld + i];
            __builtin_amdgcn_sched_barrier(0);
        } else {
#pragma unroll
            for (int u = 0; u < B; ++u) a[u] = X[(long long)in_edge[k + u < i1 ? k + u : i1 - 1] * ld + i];
        }
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (k + u < i1) v += (double)a[u];
    }
    return v;
}

template <typename T>
__device__ __forceinline__ double gather_out(const T *X, int o0, int o1, long long ld, int i)
{
    constexpr int B = 16;
    double v = 0.0;
    for (int e = o0; e < o1; e += B) {
        T a[B];
#pragma unroll
        for (int u = 0; u < B; ++u) a[u] = X[(long long)(e + u < o1 ? e + u : o1 - 1) * ld + i];
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (e + u < o1) v += (double)a[u];
    }
    return v;
}

// (F A^T)_ij = sum_{l in in(j)} F_il - sum_{l in out(j)} F_il with the out-edge sum first
// rounded to the iterate type, exactly as the edge phase stages it in Sout.
template <typename T, bool WIDE = false>
__device__ __forceinline__ double p_entry(const T *X, const int *in_edge, int i0, int i1, T sout, long long ld, int i)
{
    return gather_in<T, WIDE>(X, in_edge, i0, i1, ld, i) - (double)sout;
}

// (F A^T)_ij when the edge phase leaves the out-edge sums to the node phase (flat edge phase):
// both gathers in FP64, the in-edges first.
template <typename T, bool WIDE = false>
__device__ __forceinline__ double p_entry_flat(const T *X, const int *in_edge, int i0, int i1, int o0, int o1,
                                               long long ld, int i)
{
    return gather_in<T, WIDE>(X, in_edge, i0, i1, ld, i) - gather_out<T>(X, o0, o1, ld, i);
}

// LAT: the latency form (regular launches of instances whose F is within NODE_LATENCY_BYTES).
// Block (row block xb, node column j) of the node phase, run by NB threads: thread t owns entry
// i = xb NB + t of column j; `blk` is the block's partial index (j nxb + xb).  For NB = 64 the
// block is one wave and its sums need no barrier (the batching pool runs several such blocks of
// different instances in one workgroup).  `lds` holds 2 NB/64 doubles private to the block.
template <typename T, int NB, int UTIL, bool CHECK, bool PARTIAL, bool LAT>
__device__ __forceinline__ void node_body(const Consts &c, const Bufs<T> &b, const PartLayout &pl, int j, int xb,
                                          int blk, double *lds)
{
    constexpr int NW = NB / 64;
    const int tid = threadIdx.x & (NB - 1);
    const int i = xb * NB + tid;
    const long long ld = c.ld;
    const double beta = b.sc->beta, g = c.gamma;
    double dy2 = 0.0, p = 0.0, conj = 0.0, rnum = 0.0, rden = 0.0, nonpos = 0.0, yinf = 0.0;
    if (i < c.n) {
        const int i0 = b.in_off[j], i1 = b.in_off[j + 1];
        const long long x = (long long)j * ld + i;
        // P' = F_new A^T; V = Fbar A^T = (2/rho) P' - ((2 - rho)/rho) P
        double pn, po, y, w;
        const bool flat = c.edge_par == 2;  // the out-edge sum is gathered here too
        if (LAT) {
            // this entry's own operands first, so that their loads are in flight during the
            // gather (after the store to P the compiler could not move them above it)
            const T sout = flat ? T(0) : b.Sout[x], pot = b.P[x], yt = b.Y[x], wt = b.W[x];
            pn = flat ? p_entry_flat<T, true>(b.F, b.in_edge, i0, i1, b.out_off[j], b.out_off[j + 1], ld, i)
                      : p_entry<T, true>(b.F, b.in_edge, i0, i1, sout, ld, i);
            po = (double)pot;
            y = (double)yt;
            w = (double)wt;
            b.P[x] = (T)pn;
        } else {
            // Sout, P and W are touched once per iteration: non-temporal, like F in the edge
            // phase, so that the caches keep Y, which the edge phase reads again per edge end
            pn = flat ? p_entry_flat<T>(b.F, b.in_edge, i0, i1, b.out_off[j], b.out_off[j + 1], ld, i)
                      : p_entry<T>(b.F, b.in_edge, i0, i1, __builtin_nontemporal_load(b.Sout + x), ld, i);
            po = (double)__builtin_nontemporal_load(b.P + x);
            __builtin_nontemporal_store((T)pn, b.P + x);
            y = (double)b.Y[x];
            w = (double)__builtin_nontemporal_load(b.W + x);
        }
        const double v = fma(2.0 / c.rho, pn, -(((2.0 - c.rho) / c.rho) * po));
        const double yhat = (i != j) ? prox_dual<UTIL>(y - beta * v, beta, w, g, c.c1, -y) : 0.0;
        const T yn = (T)fma(c.rho, yhat, (1.0 - c.rho) * y);
        b.Y[x] = yn;
        if (PARTIAL) {
            const double d = (double)yn - y;
            dy2 = d * d;
        }
        if (CHECK) {
            // T = -Fhat A^T, U' = u'(T), and the pieces of p, d and rel_primal (with Y^k = y).
            const int o0 = b.out_off[j], o1 = b.out_off[j + 1];
            const double t = gather_out<T>(b.Fhat, o0, o1, ld, i) - gather_in<T>(b.Fhat, b.in_edge, i0, i1, ld, i);
            b.That[x] = t;
            double up = 0.0;
            if (i != j) {
                if (t > 0.0) {
                    up = util_du<UTIL>(t, w, g);
                    p -= util_u<UTIL>(t, w, g);
                } else {
                    nonpos = 1.0;
                }
                if (y < 0.0) {
                    conj += util_conj<UTIL>(y, w, g);
                    const double td = util_traffic<UTIL>(y, w, g) - t;
                    rnum += td * td;
                } else {
                    yinf = 1.0;
                }
                rden += t * t;
            }
            b.Up[x] = up;
        }
    }
    if (PARTIAL) {
        double zero = 0.0;
        group_sum<NW>(dy2, zero, lds);
    }
    if (CHECK) {
        group_sum<NW>(p, conj, lds);
        group_sum<NW>(rnum, rden, lds);
        group_sum<NW>(nonpos, yinf, lds);
    }
    if (tid == 0) {
        if (PARTIAL) b.part[pl.dY + blk] = dy2;
        if (CHECK) {
            b.part[pl.p + blk] = p;
            b.part[pl.conj + blk] = conj;
            b.part[pl.rnum + blk] = rnum;
            b.part[pl.rden + blk] = rden;
            b.part[pl.nonpos + blk] = nonpos;
            b.part[pl.yinf + blk] = yinf;
        }
    }
}

template <typename T, int NB, int UTIL, bool CHECK, bool PARTIAL, bool LAT>
__global__ __launch_bounds__(NB) void node_kernel(Consts c, Bufs<T> b, PartLayout pl)
{
    __shared__ double lds[2 * (NB / 64)];
    if (b.sc->stop) return;
    node_body<T, NB, UTIL, CHECK, PARTIAL, LAT>(c, b, pl, blockIdx.y, blockIdx.x, blockIdx.y * gridDim.x + blockIdx.x,
                                                lds);
}

// P = F A^T of the current F, with the out-edge sums formed in the iterate type and in the
// order the edge phase forms them, so that P is the one an uninterrupted run would hold.
template <typename T, int NB>
__global__ __launch_bounds__(NB) void p_from_f_kernel(Consts c, Bufs<T> b)
{
    const int j = blockIdx.y;
    const int i = blockIdx.x * NB + threadIdx.x;
    if (i >= c.n) return;
    const int e0 = b.out_off[j], e1 = b.out_off[j + 1];
    if (c.edge_par == 2) {  // flat edge phase: the node phase gathers both lists, as here
        b.P[(long long)j * c.ld + i] = (T)p_entry_flat<T>(b.F, b.in_edge, b.in_off[j], b.in_off[j + 1], e0, e1, c.ld, i);
        return;
    }
    T so = T(0);
    if (c.edge_par) {
        // per wave of the concurrent edge phase (edges e0 + w, e0 + w + NW, ...), then over the waves
        for (int w = 0; w < EDGE_PAR_WAVES; ++w) {
            T sw = T(0);
            for (int e = e0 + w; e < e1; e += EDGE_PAR_WAVES) sw += b.F[(long long)e * c.ld + i];
            so += sw;
        }
    } else {
        for (int e = e0; e < e1; ++e) so += b.F[(long long)e * c.ld + i];
    }
    const long long x = (long long)j * c.ld + i;
    b.P[x] = (T)p_entry<T>(b.F, b.in_edge, b.in_off[j], b.in_off[j + 1], so, c.ld, i);
}

// ----------------------------------------------------- fused node iteration
// For n <= 64*EPT <= FUSED_MAX_N one PDHG iteration is a single launch: workgroup j
// (fused_waves: 16 waves on regular iterations with up to 4 entries per lane, else 8)
// recomputes, one wave per column, the projection of every edge incident to node j (an edge
// is projected by both of its end nodes, from identical inputs with identical code, so both
// get the same bits), accumulates V[:,j] = sum_in Fbar - sum_out Fbar in registers, adds the
// waves' sums in wave order through LDS, and updates Y[:,j].  The tail's workgroup writes the edge's new F column and multiplier.  F, Y and
// mu are read from one buffer set and written to the other, so no workgroup can see a
// value of the iteration in flight.
template <int EPT, bool CHECK>
constexpr int fused_waves() { return (CHECK || EPT > 4) ? 8 : 16; }

// The body of one fused iteration for node j, run by NWV waves.  `vsh` holds
// (CHECK ? 2 : 1) * NWV * EPT * 64 doubles, `red` 2 * NWV doubles and `incs`
// FUSED_INC_CHUNK incidence entries of LDS.
// Memory latency is what bounds this body, so: the node's incidence entries are staged in
// LDS by the whole workgroup (one round trip instead of one per edge), every column load is
// unconditional (entries past n read entry 0 of the column and are then discarded), and each
// wave loads the columns of its next edge before it projects the current one.
template <typename T, int EPT, int UTIL, bool CHECK, bool PARTIAL, int NWV, bool STOPCHK>
__device__ __forceinline__ void fused_body(const Consts &c, const Bufs<T> &b, const PartLayout &pl, int parity, int j,
                                           double *vsh, double *red, int2 *incs)
{
    constexpr int RPT = (64 * EPT + 64 * NWV - 1) / (64 * NWV);  // node-phase rows per thread
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int n = c.n;
    const long long ld = c.ld;
    const T *Fc = parity ? b.F2 : b.F;
    T *Fn = parity ? b.F : b.F2;
    const T *Yc = parity ? b.Y2 : b.Y;
    T *Yn = parity ? b.Y : b.Y2;
    const double *muc = parity ? b.mu2 : b.mu;
    double *mun = parity ? b.mu : b.mu2;
    const T ta = (T)b.sc->alpha;
    const double beta = b.sc->beta, g = c.gamma, rho = c.rho, omr = 1.0 - c.rho;
    const int k0 = b.inc_off[j], k1 = b.inc_off[j + 1], deg = k1 - k0;
    const T *yj = Yc + (long long)j * ld;
    // node-phase operands (rows past n read row 0 and are never used): loaded before the edge
    // loop so that their latency overlaps it, unless they would hold more than 4 registers per
    // thread across it (small workgroups with many rows per thread), which would cost occupancy
    constexpr bool EARLY = RPT <= 2;
    T yrow[RPT], wrow[RPT];
    auto load_rows = [&]() {
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = threadIdx.x + r * 64 * NWV;
            const int ic = i < n ? i : 0;
            yrow[r] = yj[ic];
            wrow[r] = b.W[(long long)j * ld + ic];
        }
    };
    if constexpr (EARLY) load_rows();
    // column j of Y, shared by every edge incident to j (its head or its tail column)
    T yjl[EPT];
#pragma unroll
    for (int jj = 0; jj < EPT; ++jj) {
        const int i = lane + jj * 64;
        yjl[jj] = yj[i < n ? i : 0];
    }
    // the stop flag is read with the offsets, after the loads above are issued, so that no
    // round trip to memory is spent on it alone
    if (STOPCHK && (b.sc->stop | (k1 < k0))) return;
    double vacc[EPT], tacc[EPT];
#pragma unroll
    for (int jj = 0; jj < EPT; ++jj) vacc[jj] = tacc[jj] = 0.0;
    double dsum = 0.0, esum = 0.0, supsum = 0.0;
    // F[:,e] and Y[:,other end] of incidence entry x (in LDS), with the edge's c and mu
    auto fetch = [&](int x, T (&fv)[EPT], T (&yv)[EPT], double &cap, double &mu0) {
        const int2 ent = incs[x];
        const int e = ent.x, o = ent.y & 0x7fffffff;
        const T *f = Fc + (long long)e * ld;
        const T *yo = Yc + (long long)o * ld;
#pragma unroll
        for (int jj = 0; jj < EPT; ++jj) {
            const int i = lane + jj * 64;
            const int ic = i < n ? i : 0;
            fv[jj] = f[ic];
            yv[jj] = yo[ic];
        }
        cap = b.cap[e];
        mu0 = muc[e];
    };
    // One chunk of incidence entries: staged in LDS, then projected wave by wave.  The first
    // chunk (usually the only one) is a call of its own, outside any loop, so that the waits
    // the compiler places at a loop head do not hold up the loads issued above.
    auto chunk = [&](int base) {
        const int cnt = min(FUSED_INC_CHUNK, deg - base);
        if (base > 0) __syncthreads();  // the previous chunk is consumed
        for (int x = threadIdx.x; x < cnt; x += 64 * NWV) incs[x] = b.inc[k0 + base + x];
        __syncthreads();
        T fa[EPT], ya[EPT];
        double capa = 0.0, mu0a = 0.0;
        if (wv < cnt) fetch(wv, fa, ya, capa, mu0a);
    for (int idx = wv; idx < cnt; idx += NWV) {
        // the next edge of this wave (the last one again when there is none: no branch, so
        // the wait for the current edge's columns does not also wait for these loads)
        T fnx[EPT], ynx[EPT];
        double capn, mu0n;
        fetch(min(idx + NWV, cnt - 1), fnx, ynx, capn, mu0n);
        const int2 ent = incs[idx];
        const bool out = ent.y < 0;  // edge leaves j: j is its tail
        const int e = ent.x;
        const double cap = capa, mu0 = mu0a;
        T fo[EPT], q[EPT];
#pragma unroll
        for (int jj = 0; jj < EPT; ++jj) {
            const int i = lane + jj * 64;
            if (i < n) {
                fo[jj] = fa[jj];
                const T yv = ya[jj];
                q[jj] = fo[jj] + ta * (out ? yv - yjl[jj] : yjl[jj] - yv);  // Y[:,head] - Y[:,tail]
            } else {
                fo[jj] = T(0);
                q[jj] = T(-1);
            }
        }
        // the projection of Section 2.3 with the warm-started active-set search of edge_kernel:
        // comparisons in the iterate type against thresholds rounded down (exact), each lane's
        // entries added in the iterate type, lanes in FP64; support sizes by ballot
        const T thr0 = below(mu0, T(0));
        T psum = T(0), wsum = T(0);
        int cp = 0, cw = 0;
#pragma unroll
        for (int jj = 0; jj < EPT; ++jj) {
            const bool ip = q[jj] > T(0), iw = q[jj] > thr0;
            if (ip) psum += q[jj];
            if (iw) wsum += q[jj];
            cp += wave_count(ip);
            cw += wave_count(iw);
        }
        double sp = (double)psum, sw = (double)wsum;
        wave_sum2(sp, sw);
        double mu = 0.0;
        if (sp > cap) {
            mu = (sp - cap) * rcp_of(b.rcp, cp);
            int prev = cp;
            if (cw > 0) {
                const double mw = (sw - cap) * rcp_of(b.rcp, cw);
                if (mw > mu) {
                    mu = mw;
                    prev = mw >= mu0 ? cw : 0x7fffffff;
                }
            }
            // each pass counts the support first; only a support that shrank needs its sum
            for (int pass = 0; pass <= n; ++pass) {
                const T thr = below(mu, T(0));
                int cnt = 0;
#pragma unroll
                for (int jj = 0; jj < EPT; ++jj) cnt += wave_count(q[jj] > thr);
                if (cnt >= prev) break;
                T ps = T(0);
#pragma unroll
                for (int jj = 0; jj < EPT; ++jj)
                    if (q[jj] > thr) ps += q[jj];
                const double s = wave_sum((double)ps);
                mu = (s - cap) * rcp_of(b.rcp, cnt);
                prev = cnt;
            }
        }
        // Fhat, Fbar and the relaxed F in the iterate type (V and the partials add in FP64)
        double gmax = -INFINITY;
        const T mut = (T)mu, rhot = (T)rho, omrt = (T)omr;
#pragma unroll
        for (int jj = 0; jj < EPT; ++jj) {
            const int i = lane + jj * 64;
            if (i < n) {
                const T fh = q[jj] > mut ? q[jj] - mut : T(0);
                const T fb = T(2) * fh - fo[jj];
                vacc[jj] += (double)(out ? -fb : fb);
                if (CHECK) tacc[jj] += (double)(out ? fh : -fh);  // T = -Fhat A^T
                if (out) {
                    const T fn = rhot * fh + omrt * fo[jj];
                    // non-temporal: this launch reads F (both ends' loads) only from the other
                    // buffer, so the new column need not take cache room from them
                    __builtin_nontemporal_store(fn, Fn + (long long)e * ld + i);
                    if (PARTIAL) {
                        const double d = (double)fn - (double)fo[jj];
                        dsum += d * d;
                    }
                    if (CHECK) {
                        b.Fhat[(long long)e * ld + i] = fh;
                        const T dd = fh - q[jj];
                        b.D[(long long)e * ld + i] = dd;
                        esum += (double)dd * (double)dd;
                        gmax = fmax(gmax, (double)(ya[jj] - yjl[jj]));  // (Y A)_il of the leaving edge
                    }
                }
            }
        }
        if (out) {
            if (lane == 0) mun[e] = mu;
            if (CHECK) supsum += cap * fmax(wave_max(gmax), 0.0);  // c_l (max_i (Y A)_il)_+
        }
#pragma unroll
        for (int jj = 0; jj < EPT; ++jj) {
            fa[jj] = fnx[jj];
            ya[jj] = ynx[jj];
        }
        capa = capn;
        mu0a = mu0n;
    }
    };
    chunk(0);
    for (int base = FUSED_INC_CHUNK; base < deg; base += FUSED_INC_CHUNK) chunk(base);
    if constexpr (!EARLY) load_rows();
#pragma unroll
    for (int jj = 0; jj < EPT; ++jj) {
        vsh[(wv * EPT + jj) * 64 + lane] = vacc[jj];
        if (CHECK) vsh[NWV * EPT * 64 + (wv * EPT + jj) * 64 + lane] = tacc[jj];
    }
    __syncthreads();
    double dy2 = 0.0, p = 0.0, conj = 0.0, rnum = 0.0, rden = 0.0, nonpos = 0.0, yinf = 0.0;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int i = threadIdx.x + r * 64 * NWV;
        if (i >= n) continue;
        const int jj = i >> 6, L = i & 63;
        double v = 0.0, t = 0.0;
#pragma unroll
        for (int w = 0; w < NWV; ++w) {
            v += vsh[(w * EPT + jj) * 64 + L];
            if (CHECK) t += vsh[NWV * EPT * 64 + (w * EPT + jj) * 64 + L];
        }
        const long long x = (long long)j * ld + i;
        const double y = (double)yrow[r], w = (double)wrow[r];
        const double yhat = (i != j) ? prox_dual<UTIL>(y - beta * v, beta, w, g, c.c1, -y) : 0.0;
        const T yn = (T)fma(rho, yhat, omr * y);
        Yn[x] = yn;
        if (PARTIAL) {
            const double d = (double)yn - y;
            dy2 += d * d;
        }
        if (CHECK) {
            b.That[x] = t;
            double up = 0.0;
            if (i != j) {
                if (t > 0.0) {
                    up = util_du<UTIL>(t, w, g);
                    p -= util_u<UTIL>(t, w, g);
                } else {
                    nonpos += 1.0;
                }
                if (y < 0.0) {
                    conj += util_conj<UTIL>(y, w, g);
                    const double td = util_traffic<UTIL>(y, w, g) - t;
                    rnum += td * td;
                } else {
                    yinf += 1.0;
                }
                rden += t * t;
            }
            b.Up[x] = up;
        }
    }
    if (PARTIAL) group_sum<NWV>(dsum, dy2, red);
    if (CHECK) {
        double sup = lane == 0 ? supsum : 0.0;  // supsum is uniform within a wave
        group_sum<NWV>(esum, sup, red);
        supsum = sup;
        group_sum<NWV>(p, conj, red);
        group_sum<NWV>(rnum, rden, red);
        group_sum<NWV>(nonpos, yinf, red);
    }
    if (threadIdx.x == 0) {
        if (PARTIAL) {
            b.part[pl.dF + j] = dsum;
            b.part[pl.dY + j] = dy2;
        }
        if (CHECK) {
            b.part[pl.e + j] = esum;
            b.part[pl.sup + j] = supsum;
            b.part[pl.p + j] = p;
            b.part[pl.conj + j] = conj;
            b.part[pl.rnum + j] = rnum;
            b.part[pl.rden + j] = rden;
            b.part[pl.nonpos + j] = nonpos;
            b.part[pl.yinf + j] = yinf;
        }
    }
}

template <typename T, int EPT, int UTIL, bool CHECK, bool PARTIAL>
__global__ __launch_bounds__((64 * fused_waves<EPT, CHECK>())) void fused_kernel(Consts c, Bufs<T> b, PartLayout pl,
                                                                               int parity)
{
    constexpr int NWV = fused_waves<EPT, CHECK>();
    extern __shared__ double vsh[];
    __shared__ double red[2 * NWV];
    __shared__ int2 incs[FUSED_INC_CHUNK];
    fused_body<T, EPT, UTIL, CHECK, PARTIAL, NWV, true>(c, b, pl, parity, (int)blockIdx.x, vsh, red, incs);
}

// ---------------------------------------------------------- residual pass
// Per edge: G[:,l] = U'[:,head] - U'[:,tail]; ||G_l||^2 and <G_l, D_l>.  One wave per edge,
// RES_EDGES consecutive edges per block; the block adds its edges' values in edge order and
// writes one partial per block.
template <typename T>
__device__ __forceinline__ void residual_edge(const Consts &c, const Bufs<T> &b, int e, double &a, double &bb)
{
    const int lane = threadIdx.x & 63;
    const long long ld = c.ld;
    const double *uh = b.Up + (long long)__builtin_amdgcn_readfirstlane(b.head[e]) * ld;
    const double *ut = b.Up + (long long)__builtin_amdgcn_readfirstlane(b.tail[e]) * ld;
    const T *d = b.D + (long long)e * ld;
    a = 0.0;
    bb = 0.0;
    // four rows per lane and pass, loaded unconditionally (rows past n read row 0 and are
    // discarded) so that the twelve loads of a pass are in flight together
    for (int i0 = lane; i0 < c.n; i0 += 256) {
        double h4[4], t4[4], d4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + 64 * u, ic = i < c.n ? i : 0;
            h4[u] = uh[ic];
            t4[u] = ut[ic];
            d4[u] = (double)d[ic];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i0 + 64 * u < c.n) {
                const double gg = h4[u] - t4[u];
                a += gg * gg;
                bb += gg * d4[u];
            }
    }
    a = wave_sum(a);
    bb = wave_sum(bb);
}

// Block `blk` of the residual pass (RES_EDGES waves); `lds` holds 2 * RES_EDGES doubles.
template <typename T>
__device__ __forceinline__ void residual_body(const Consts &c, const Bufs<T> &b, const PartLayout &pl, int blk,
                                              double *lds)
{
    const int w = threadIdx.x >> 6, e = blk * RES_EDGES + w;
    double a = 0.0, bb = 0.0;
    if (e < c.m) residual_edge<T>(c, b, e, a, bb);
    if ((threadIdx.x & 63) == 0) {
        lds[w] = a;
        lds[RES_EDGES + w] = bb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
        for (int x = 0; x < RES_EDGES; ++x) {
            sa += lds[x];
            sb += lds[RES_EDGES + x];
        }
        b.part[pl.a + blk] = sa;
        b.part[pl.b + blk] = sb;
    }
}

template <typename T>
__global__ __launch_bounds__(64 * RES_EDGES) void residual_kernel(Consts c, Bufs<T> b, PartLayout pl)
{
    __shared__ double lds[2 * RES_EDGES];
    if (b.sc->stop) return;
    const int items = c.nrp;
    const int blk = xcd_item(blockIdx.x, items);
    if (blk >= items) return;
    residual_body<T>(c, b, pl, blk, lds);
}

// ----------------------------------------------------------------- control
constexpr int CTRL_BLOCK = 512;
constexpr int NQ = CTRL_NQ;  // reduced quantities

// The partial segments of the control and their lengths (dF and dY first: a control without a
// check reduces only those two).
__device__ __forceinline__ void control_segments(const Consts &c, const PartLayout &pl, long long (&seg)[NQ],
                                                 long long (&len)[NQ])
{
    const long long s[NQ] = {pl.dF, pl.dY, pl.e, pl.sup, pl.a, pl.b, pl.p, pl.conj, pl.rnum, pl.rden, pl.nonpos,
                             pl.yinf};
    const long long l[NQ] = {c.nep, c.nnp, c.nep, c.nep, c.nrp, c.nrp, c.nnp, c.nnp, c.nnp, c.nnp, c.nnp, c.nnp};
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        seg[q] = s[q];
        len[q] = l[q];
    }
}

// Sums, over the CTRL_BLOCK threads of a workgroup, the entries x0 <= x < x1 of the first nq
// segments (each only up to its length): one thread-strided pass with all loads independent, then
// wave sums and the CTRL_BLOCK/64 wave totals added in wave order.  `lds` holds NQ * CTRL_BLOCK/64
// doubles; the totals are valid in thread 0.
__device__ __forceinline__ void block_sums(const double *P, const long long (&seg)[NQ], const long long (&len)[NQ],
                                           int nq, long long x0, long long x1, double (&tot)[NQ], double *lds)
{
    constexpr int NW = CTRL_BLOCK / 64;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    // every load is unconditional (an index past its segment reads the segment's first entry,
    // which is then discarded), so that the NQ loads of a pass are in flight together
#pragma unroll 2
    for (long long x = x0 + threadIdx.x; x < x1; x += CTRL_BLOCK) {
        double v[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = P[seg[q] + (x < len[q] ? x : 0)];
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] += (q < nq && x < len[q]) ? v[q] : 0.0;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double t = wave_sum(acc[q]);
        if (lane == 0) lds[q * NW + wid] = t;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double t = 0.0;
        for (int w = 0; w < NW; ++w) t += lds[q * NW + w];
        tot[q] = t;
    }
}

// First level of a split control reduction: workgroup g sums entries [g * chunk, (g + 1) * chunk)
// of every segment into red[q * CTRL_GROUPS + g], chunk = ceil(longest / CTRL_GROUPS).
template <typename T>
__global__ __launch_bounds__(CTRL_BLOCK) void control_split_kernel(Consts c, Bufs<T> b, PartLayout pl, int check)
{
    __shared__ double lds[NQ * (CTRL_BLOCK / 64)];
    if (b.sc->stop) return;
    long long seg[NQ], len[NQ];
    control_segments(c, pl, seg, len);
    const int nq = check ? NQ : 2;
    long long most = 0;
    for (int q = 0; q < nq; ++q) most = len[q] > most ? len[q] : most;
    const long long chunk = (most + CTRL_GROUPS - 1) / CTRL_GROUPS;
    const long long x0 = (long long)blockIdx.x * chunk, x1 = x0 + chunk < most ? x0 + chunk : most;
    double tot[NQ];
    block_sums(b.part, seg, len, nq, x0, x1, tot, lds);
    if (threadIdx.x == 0)
        for (int q = 0; q < nq; ++q) b.part[pl.red + (long long)q * CTRL_GROUPS + blockIdx.x] = tot[q];
}

// The control: totals of the partial segments (or, with `split`, of the first-level sums that
// control_split_kernel left), then the residuals, the stop test and the primal weight.  Run by
// one CTRL_BLOCK-thread block; `lds` holds NQ * CTRL_BLOCK/64 doubles.
template <typename T>
__device__ __forceinline__ void control_body(const Consts &c, const Bufs<T> &b, const PartLayout &pl, int check,
                                             int adapt, long long k_after, double *lds, bool split = false)
{
    DevScalars *sc = b.sc;
    long long seg[NQ], len[NQ];
    control_segments(c, pl, seg, len);
    if (split) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            seg[q] = pl.red + (long long)q * CTRL_GROUPS;
            len[q] = CTRL_GROUPS;
        }
    }
    const int nq = check ? NQ : 2;
    long long most = 0;
    for (int q = 0; q < nq; ++q) most = len[q] > most ? len[q] : most;
    double tot[NQ];
    block_sums(b.part, seg, len, nq, 0, most, tot, lds);
    if (threadIdx.x != 0) return;
    const double dF2 = tot[0], dY2 = tot[1], e = tot[2], sup = tot[3], a = tot[4], bb = tot[5], psum = tot[6],
                 conj = tot[7], rnum = tot[8], rden = tot[9], nonpos = tot[10], yinf = tot[11];
    const double dF = sqrt(dF2), dY = sqrt(dY2);
    sc->dF = dF;
    sc->dY = dY;
    bool converged = false;
    if (check) {
        const double n = c.n, m = c.m;
        const bool tfeas = nonpos == 0.0, yfeas = yinf == 0.0;
        double r = INFINITY, p = INFINITY, reld = INFINITY;
        if (tfeas) {
            // eq. (e-res)
            r = (e > 0.0 && bb >= 0.0) ? a - bb * bb / e : a;
            p = psum;
            reld = a > 0.0 ? sqrt(fmax(r, 0.0) / a) : INFINITY;
        }
        double d = -INFINITY, relp = INFINITY;
        if (yfeas) {
            d = -conj - sup;  // dual objective of the reduced Lagrangian (e-L)
            relp = rden > 0.0 ? sqrt(rnum) / sqrt(rden) : INFINITY;
        }
        const double relg = (isfinite(p) && isfinite(d)) ? (p - d) / (1.0 + fabs(p) + fabs(d)) : INFINITY;
        double kkt = INFINITY;
        if (tfeas && yfeas) kkt = fmax(relp, fmax(reld, relg));
        sc->r = r;
        sc->r_paper = r / (n * m);
        sc->rel_primal = relp;
        sc->rel_dual = reld;
        sc->rel_gap = relg;
        sc->rel_kkt = kkt;
        sc->primal_obj = p;
        sc->dual_obj = d;
        sc->infeasible_frac = nonpos / (n * (n - 1.0));
        sc->a = a;
        sc->b = bb;
        sc->e = e;
        sc->checked = 1;
        converged = c.stop_rule == 0 ? (kkt <= c.tol) : (r < n * m * c.tol);
    } else {
        sc->checked = 0;
    }
    const bool bad = !isfinite(dF) || !isfinite(dY);
    // Algorithm 2.1 step 3, (e-primal_weight)
    if (!bad && adapt && dF > c.tau && dY > c.tau) {
        const double om = pow(dY / dF, c.theta) * pow(sc->omega, 1.0 - c.theta);
        sc->omega = om;
        sc->alpha = sc->eta / om;
        sc->beta = sc->eta * om;
    }
    sc->k = k_after;
    if (bad) {
        sc->state = 3;
        sc->stop = 1;
    } else if (converged && sc->stop_enabled) {
        sc->state = 1;
        sc->stop = 1;
    }
}

// k_inc: iterations since the previous control launch, so that a captured block of iterations
// carries no absolute iteration number (the count is read before control_body's barriers, and
// only thread 0 writes it back after them).
template <typename T>
__global__ __launch_bounds__(CTRL_BLOCK) void control_kernel(Consts c, Bufs<T> b, PartLayout pl, int check,
                                                              int adapt, long long k_inc, int split)
{
    __shared__ double lds[NQ * (CTRL_BLOCK / 64)];
    if (b.sc->stop) return;
    const long long k_after = b.sc->k + k_inc;
    control_body<T>(c, b, pl, check, adapt, k_after, lds, split != 0);
}

template <typename T>
__global__ void poison_kernel(Bufs<T> b, int which, long long off)
{
    if (which == 0) b.F[off] = (T)NAN;
    else b.Y[off] = (T)NAN;
}

// ------------------------------------------------------------------- pool
// Batched iteration of many instances (each with n <= FUSED_MAX_N): one launch per
// iteration covers every node of every active slot.  A slot's iteration count, buffer
// parity and adapt schedule follow from the pool's iteration counter G and the values
// recorded at admission, so nothing per slot is written by the host between launches.
template <typename T>
__device__ __forceinline__ bool slot_live(const SlotDesc<T> &d, long long G, long long &k)
{
    if (!d.active || d.b.sc->stop) return false;
    k = d.k0 + (G - d.G0);
    return k < d.max_iter;
}

// CHECK is uniform over a launch (every slot checks at the same pool iteration), so the
// check variant is a kernel of its own and the register count of the regular kernel stays low.
template <typename T, int EPT, int UTIL, bool CHECK, int NWV>
__device__ __forceinline__ void pool_body(const SlotDesc<T> &d, int parity, int j, bool partial, double *vsh,
                                          double *red, int2 *incs)
{
    // the slot's stop flag was read by slot_live
    if (CHECK) fused_body<T, EPT, UTIL, true, true, NWV, false>(d.c, d.b, d.pl, parity, j, vsh, red, incs);
    else if (partial)
        fused_body<T, EPT, UTIL, false, true, NWV, false>(d.c, d.b, d.pl, parity, j, vsh, red, incs);
    else fused_body<T, EPT, UTIL, false, false, NWV, false>(d.c, d.b, d.pl, parity, j, vsh, red, incs);
}

template <typename T, int EPT, bool CHECK, int NWV>
__device__ __forceinline__ void pool_util(const SlotDesc<T> &d, int parity, int j, bool partial, double *vsh,
                                          double *red, int2 *incs)
{
    if (d.c.utility == 0) pool_body<T, EPT, 0, CHECK, NWV>(d, parity, j, partial, vsh, red, incs);
    else if (d.c.utility == 1) pool_body<T, EPT, 1, CHECK, NWV>(d, parity, j, partial, vsh, red, incs);
    else pool_body<T, EPT, 2, CHECK, NWV>(d, parity, j, partial, vsh, red, incs);
}

// Iteration G + it of the pool: workgroup b runs the fused body of work item b = (slot, node j)
// with NWV waves.  The grid is the item count rounded up (so that a captured step fits every
// count up to its grid); workgroups past the count read from the pool state return at once.
// The dynamic LDS holds the V (and T) sums of NWV waves at the largest entries per lane the
// pool admits.
template <typename T, int NWV, bool CHECK>
__global__ __launch_bounds__(64 * NWV) void pool_fused_kernel(const SlotDesc<T> *slots, const int2 *work,
                                                              const PoolState *ps, int it)
{
    extern __shared__ double vsh[];
    __shared__ double red[2 * NWV];
    __shared__ int2 incs[FUSED_INC_CHUNK];
    if ((int)blockIdx.x >= ps->nwork) return;
    const long long G = ps->G + it;
    const int2 wk = work[blockIdx.x];
    const SlotDesc<T> &d = slots[wk.x];
    long long k;
    if (!slot_live(d, G, k)) return;
    const int parity = d.par0 ^ (int)((G - d.G0) & 1);
    const bool partial = CHECK || adapts_at(d.c, k);
    const int n = d.c.n;
    if (n <= 64) pool_util<T, 1, CHECK, NWV>(d, parity, wk.y, partial, vsh, red, incs);
    else if (n <= 128) pool_util<T, 2, CHECK, NWV>(d, parity, wk.y, partial, vsh, red, incs);
    else if (n <= 256) pool_util<T, 4, CHECK, NWV>(d, parity, wk.y, partial, vsh, red, incs);
    else pool_util<T, 8, CHECK, NWV>(d, parity, wk.y, partial, vsh, red, incs);
}

// Two-phase slots of the pool.  Edge launch: workgroup b is flat edge item b = (slot, block of
// EDGE_PAR_WAVES edges), one wave per edge (the flat edge phase of a single solve).
template <typename T, int NV, bool CHECK>
__device__ __forceinline__ void pool_flat(const SlotDesc<T> &d, int blk, bool partial, double *red)
{
    if (CHECK) flat_block<T, NV, true, true>(d.c, d.b, d.pl, blk, red);
    else if (partial) flat_block<T, NV, false, true>(d.c, d.b, d.pl, blk, red);
    else flat_block<T, NV, false, false>(d.c, d.b, d.pl, blk, red);
}

template <typename T, bool CHECK>
__global__ __launch_bounds__(64 * EDGE_PAR_WAVES) void pool_edge_kernel(const SlotDesc<T> *slots, const int2 *ework,
                                                                        const PoolState *ps, int it)
{
    __shared__ double red[3 * EDGE_PAR_WAVES];
    if ((int)blockIdx.x >= ps->nedge) return;
    const int2 wk = ework[blockIdx.x];
    const SlotDesc<T> &d = slots[wk.x];
    long long k;
    if (!slot_live(d, ps->G + it, k)) return;
    const bool partial = CHECK || adapts_at(d.c, k);
    if (d.c.edge_ept == 1) pool_flat<T, 1, CHECK>(d, wk.y, partial, red);
    else if (d.c.edge_ept == 2) pool_flat<T, 2, CHECK>(d, wk.y, partial, red);
    else pool_flat<T, 4, CHECK>(d, wk.y, partial, red);
}

// Node launch: each wave of a workgroup is node item (slot, j * ceil(n/64) + xb): rows
// 64 xb .. 64 xb + 63 of column j, the node phase of a single solve with 64-thread blocks (wave
// sums only, no barrier), in its latency form, which computes the same values as the streaming
// form.  Waves past the item count return at once.
template <typename T, int UTIL, bool CHECK>
__device__ __forceinline__ void pool_node_util(const SlotDesc<T> &d, int j, int xb, int blk, bool partial)
{
    if (CHECK) node_body<T, 64, UTIL, true, true, false>(d.c, d.b, d.pl, j, xb, blk, nullptr);
    else if (partial) node_body<T, 64, UTIL, false, true, false>(d.c, d.b, d.pl, j, xb, blk, nullptr);
    else node_body<T, 64, UTIL, false, false, true>(d.c, d.b, d.pl, j, xb, blk, nullptr);
}

template <typename T, bool CHECK>
__global__ __launch_bounds__(64 * POOL_NODE_WAVES) void pool_node_kernel(const SlotDesc<T> *slots, const int2 *nwork,
                                                                         const PoolState *ps, int it)
{
    const int item = (int)blockIdx.x * POOL_NODE_WAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (item >= ps->nnode) return;
    const int2 wk = nwork[item];
    const SlotDesc<T> &d = slots[wk.x];
    long long k;
    if (!slot_live(d, ps->G + it, k)) return;
    const bool partial = CHECK || adapts_at(d.c, k);
    const int nxb = (d.c.n + 63) / 64;
    const int j = wk.y / nxb, xb = wk.y - j * nxb;
    if (d.c.utility == 0) pool_node_util<T, 0, CHECK>(d, j, xb, wk.y, partial);
    else if (d.c.utility == 1 && d.c.c1 == 1.0) pool_node_util<T, UTIL_POWER_HALF, CHECK>(d, j, xb, wk.y, partial);
    else if (d.c.utility == 1) pool_node_util<T, 1, CHECK>(d, j, xb, wk.y, partial);
    else pool_node_util<T, 2, CHECK>(d, j, xb, wk.y, partial);
}

// Residual pass of every slot: workgroup b is block b - res_off[s] of slot s, where res_off
// (nslots + 1 entries, nondecreasing) counts the residual blocks of the slots before s.
template <typename T>
__global__ __launch_bounds__(64 * RES_EDGES) void pool_residual_kernel(const SlotDesc<T> *slots, const int *res_off,
                                                                       const PoolState *ps, int nslots, int it)
{
    __shared__ double lds[2 * RES_EDGES];
    const int item = blockIdx.x;
    if (item >= ps->nres) return;
    int lo = 0, hi = nslots;  // the last slot s with res_off[s] <= item
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (res_off[mid] <= item) lo = mid;
        else hi = mid;
    }
    const SlotDesc<T> &d = slots[lo];
    long long k;
    if (!slot_live(d, ps->G + it, k)) return;
    residual_body<T>(d.c, d.b, d.pl, item - res_off[lo], lds);
}

// one block per slot; acts on the slots whose iteration G + it adapted omega or was checked
template <typename T>
__global__ __launch_bounds__(CTRL_BLOCK) void pool_control_kernel(const SlotDesc<T> *slots, const PoolState *ps,
                                                                  int it, int check)
{
    __shared__ double lds[NQ * (CTRL_BLOCK / 64)];
    const SlotDesc<T> &d = slots[blockIdx.x];
    long long k;
    if (!slot_live(d, ps->G + it, k)) return;
    const bool adapt = adapts_at(d.c, k);
    if (!check && !adapt) return;
    control_body<T>(d.c, d.b, d.pl, check, adapt, k + 1, lds);
}

// Copies every slot's scalar record into one array (one host copy per step) and advances the
// pool's iteration counter past the step (the last launch of a step: none of its launches
// reads G after this one starts).
template <typename T>
__global__ void pool_gather_kernel(const SlotDesc<T> *slots, int nslots, DevScalars *out, PoolState *ps, int iters)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nslots && slots[s].active) out[s] = *slots[s].b.sc;
    if (s == 0) ps->G += iters;
}

// ---------------------------------------------------------------- launchers
// A launch that records the timing events e0/e1 with its own dispatch when they are given, else
// a plain launch (the form a captured graph takes).
#define MCF_LAUNCH(kern, grid, block, lds, st, e0, e1, flags, ...)                                \
    do {                                                                                       \
        if ((e0) || (e1)) hipExtLaunchKernelGGL(kern, grid, block, lds, st, e0, e1, flags, __VA_ARGS__); \
        else hipLaunchKernelGGL(kern, grid, block, lds, st, __VA_ARGS__);                       \
    } while (0)

// Two-phase edge launch shapes compiled below, per iterate size.  Up to n = 64 * 8 * VEC (2048
// FP32, 1024 FP64) a column fits one wave with at most 8 vectors per lane, and a tail's
// out-edges can be projected concurrently.  Beyond that a tail's waves share each column: each
// lane holds 2 * NV * VEC iterate values (F and q), with the out-edge sums in LDS; 8 waves per
// column keep that near 100 VGPRs, 16 for the largest FP64 columns.  {1, nv, 1}: edge_kernel_par
// (one wave per out-edge, columns of up to 64 nv vec entries); {wpe, nv, 0}: edge_kernel with
// wpe waves per column of up to 64 wpe nv vec entries, the out-edges of a tail in turn;
// {1, nv, 2}: edge_kernel_flat, one wave per edge over a flat grid of edges (columns of up to
// 64 nv vec entries), the out-edge sums gathered by the node phase.
static const EdgeShape EDGE_SHAPES_F32[] = {{1, 1, 1}, {1, 2, 1}, {1, 4, 1}, {1, 8, 1}, {1, 1, 2}, {1, 2, 2},
                                            {1, 4, 2}, {1, 8, 2}, {4, 1, 0}, {4, 2, 0}, {4, 4, 0}, {8, 3, 0},
                                            {8, 4, 0}, {8, 6, 0}, {8, 8, 0}};
static const EdgeShape EDGE_SHAPES_F64[] = {{1, 1, 1}, {1, 2, 1}, {1, 4, 1}, {1, 8, 1}, {1, 1, 2}, {1, 2, 2},
                                            {1, 4, 2}, {1, 8, 2}, {4, 1, 0}, {4, 2, 0}, {4, 4, 0}, {8, 4, 0},
                                            {8, 8, 0}, {16, 8, 0}};

int edge_shape_list(int bytes, const EdgeShape **list)
{
    if (bytes == 4) {
        *list = EDGE_SHAPES_F32;
        return (int)(sizeof(EDGE_SHAPES_F32) / sizeof(EdgeShape));
    }
    *list = EDGE_SHAPES_F64;
    return (int)(sizeof(EDGE_SHAPES_F64) / sizeof(EdgeShape));
}

bool edge_shape_valid(EdgeShape sh, int n, int bytes)
{
    const EdgeShape *list;
    const int cnt = edge_shape_list(bytes, &list);
    for (int x = 0; x < cnt; ++x)
        if (list[x].wpe == sh.wpe && list[x].ept == sh.ept && list[x].par == sh.par)
            return n <= 64 * sh.wpe * (16 / bytes) * sh.ept;
    return false;
}

// Shapes picked by measurement: the table is written by paper_2501_17996_amd/tune.py, which
// times every compiled shape and node block on the GPU at a ladder of sizes.  Entries are
// ascending in n_max per iterate size; an entry applies to every n up to its n_max above the
// previous one's.  The choice depends on (n, iterate size) only, so results stay deterministic.
struct TunedEntry {
    int bytes, n_max;
    EdgeShape sh;
    int node_block;
};
#include "tuned_shapes.inc"

static const TunedEntry *tuned_for(int n, int bytes)
{
    for (const TunedEntry &t : TUNED_SHAPES)
        if (t.bytes == bytes && n <= t.n_max) return &t;
    return nullptr;
}

// Without a table entry: the smallest shape whose columns cover n.
static EdgeShape edge_shape_default(int n, int bytes)
{
    const int vec = 16 / bytes;
    const int nvp[] = {1, 2, 4, 8};
    for (int nv : nvp)
        if (n <= 64 * vec * nv) return {1, nv, 1};
    const int nv4[] = {1, 2, 4};
    for (int nv : nv4)
        if (n <= 256 * vec * nv) return {4, nv, 0};
    if (bytes == 4) {
        const int nv8[] = {3, 4, 6, 8};
        for (int nv : nv8)
            if (n <= 512 * vec * nv) return {8, nv, 0};
        return {8, 8, 0};
    }
    if (n <= 512 * vec * 4) return {8, 4, 0};
    if (n <= 512 * vec * 8) return {8, 8, 0};
    return {16, 8, 0};
}

EdgeShape edge_shape_for(int n, int bytes)
{
    const TunedEntry *t = tuned_for(n, bytes);
    if (t && edge_shape_valid(t->sh, n, bytes)) return t->sh;
    return edge_shape_default(n, bytes);
}

int node_block_for(int n, int bytes)
{
    const TunedEntry *t = tuned_for(n, bytes);
    if (t && (t->node_block == 64 || t->node_block == 256)) return t->node_block;
    return n <= 512 ? 64 : 256;
}

template <typename T>
hipError_t launch_init(const Consts &c, const Bufs<T> &b, double omega0, hipStream_t st)
{
    hipLaunchKernelGGL(init_kernel<T>, dim3(1024), dim3(256), 0, st, c, b, omega0);
    return hipGetLastError();
}

template <typename T, int WPE, int NV>
static void edge_go(const Consts &c, const Bufs<T> &b, const PartLayout &pl, bool check, bool partial,
                    hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    const dim3 grid(xcd_grid(WPE == 1 ? (c.n + 3) / 4 : c.n)), block(WPE == 1 ? 256 : 64 * WPE);
    if (check)
        MCF_LAUNCH((edge_kernel<T, WPE, NV, true, true>), grid, block, 0, st, e0, e1, 0, c, b, pl);
    else if (partial)
        MCF_LAUNCH((edge_kernel<T, WPE, NV, false, true>), grid, block, 0, st, e0, e1, 0, c, b, pl);
    else
        MCF_LAUNCH((edge_kernel<T, WPE, NV, false, false>), grid, block, 0, st, e0, e1, 0, c, b, pl);
}

template <typename T, int NV>
static void edge_par_go(const Consts &c, const Bufs<T> &b, const PartLayout &pl, bool check, bool partial,
                        hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    const dim3 grid(xcd_grid(c.n)), block(64 * EDGE_PAR_WAVES);
    if (check)
        MCF_LAUNCH((edge_kernel_par<T, NV, true, true>), grid, block, 0, st, e0, e1, 0, c, b, pl);
    else if (partial)
        MCF_LAUNCH((edge_kernel_par<T, NV, false, true>), grid, block, 0, st, e0, e1, 0, c, b, pl);
    else
        MCF_LAUNCH((edge_kernel_par<T, NV, false, false>), grid, block, 0, st, e0, e1, 0, c, b, pl);
}

template <typename T, int NV>
static void edge_flat_go(const Consts &c, const Bufs<T> &b, const PartLayout &pl, bool check, bool partial,
                         hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    const dim3 grid(xcd_grid(c.nep)), block(64 * EDGE_PAR_WAVES);
    if (check)
        MCF_LAUNCH((edge_kernel_flat<T, NV, true, true>), grid, block, 0, st, e0, e1, 0, c, b, pl);
    else if (partial)
        MCF_LAUNCH((edge_kernel_flat<T, NV, false, true>), grid, block, 0, st, e0, e1, 0, c, b, pl);
    else
        MCF_LAUNCH((edge_kernel_flat<T, NV, false, false>), grid, block, 0, st, e0, e1, 0, c, b, pl);
}

template <typename T>
hipError_t launch_edge(const Consts &c, const Bufs<T> &b, const PartLayout &pl, EdgeShape sh, bool check,
                       bool partial, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    if (sh.par == 2) {
        switch (sh.ept) {
        case 1: edge_flat_go<T, 1>(c, b, pl, check, partial, st, e0, e1); return hipGetLastError();
        case 2: edge_flat_go<T, 2>(c, b, pl, check, partial, st, e0, e1); return hipGetLastError();
        case 4: edge_flat_go<T, 4>(c, b, pl, check, partial, st, e0, e1); return hipGetLastError();
        case 8: edge_flat_go<T, 8>(c, b, pl, check, partial, st, e0, e1); return hipGetLastError();
        default: return hipErrorInvalidValue;
        }
    }
    if (sh.par) {
        switch (sh.ept) {
        case 1: edge_par_go<T, 1>(c, b, pl, check, partial, st, e0, e1); return hipGetLastError();
        case 2: edge_par_go<T, 2>(c, b, pl, check, partial, st, e0, e1); return hipGetLastError();
        case 4: edge_par_go<T, 4>(c, b, pl, check, partial, st, e0, e1); return hipGetLastError();
        case 8: edge_par_go<T, 8>(c, b, pl, check, partial, st, e0, e1); return hipGetLastError();
        default: return hipErrorInvalidValue;
        }
    }
#define MCF_EDGE_CASE(W, V) \
    if (sh.wpe == W && sh.ept == V) { edge_go<T, W, V>(c, b, pl, check, partial, st, e0, e1); return hipGetLastError(); }
    MCF_EDGE_CASE(4, 1)
    MCF_EDGE_CASE(4, 2)
    MCF_EDGE_CASE(4, 4)
    MCF_EDGE_CASE(8, 4)
    MCF_EDGE_CASE(8, 8)
    if constexpr (sizeof(T) == 4) {
        MCF_EDGE_CASE(8, 3)
        MCF_EDGE_CASE(8, 6)
    } else {
        MCF_EDGE_CASE(16, 8)
    }
#undef MCF_EDGE_CASE
    return hipErrorInvalidValue;
}

template <typename T, int NB, int UTIL>
static void node_go(const Consts &c, const Bufs<T> &b, const PartLayout &pl, bool check, bool partial, hipStream_t st,
                    hipEvent_t e0, hipEvent_t e1)
{
    const dim3 grid((c.n + NB - 1) / NB, c.n);
    if (check) MCF_LAUNCH((node_kernel<T, NB, UTIL, true, true, false>), grid, dim3(NB), 0, st, e0, e1, 0, c, b, pl);
    else if (partial) MCF_LAUNCH((node_kernel<T, NB, UTIL, false, true, false>), grid, dim3(NB), 0, st, e0, e1, 0, c, b, pl);
    else if (c.node_latency) MCF_LAUNCH((node_kernel<T, NB, UTIL, false, false, true>), grid, dim3(NB), 0, st, e0, e1, 0, c, b, pl);
    else MCF_LAUNCH((node_kernel<T, NB, UTIL, false, false, false>), grid, dim3(NB), 0, st, e0, e1, 0, c, b, pl);
}

template <typename T>
hipError_t launch_node(const Consts &c, const Bufs<T> &b, const PartLayout &pl, bool check, bool partial,
                       hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    // gamma = 1/2 (c1 = gamma / (1 - gamma) = 1) takes the kernels compiled for it
    const bool half = c.utility == 1 && c.c1 == 1.0;
    if (c.node_block == 64) {
        if (c.utility == 0) node_go<T, 64, 0>(c, b, pl, check, partial, st, e0, e1);
        else if (half) node_go<T, 64, UTIL_POWER_HALF>(c, b, pl, check, partial, st, e0, e1);
        else if (c.utility == 1) node_go<T, 64, 1>(c, b, pl, check, partial, st, e0, e1);
        else node_go<T, 64, 2>(c, b, pl, check, partial, st, e0, e1);
    } else {
        if (c.utility == 0) node_go<T, 256, 0>(c, b, pl, check, partial, st, e0, e1);
        else if (half) node_go<T, 256, UTIL_POWER_HALF>(c, b, pl, check, partial, st, e0, e1);
        else if (c.utility == 1) node_go<T, 256, 1>(c, b, pl, check, partial, st, e0, e1);
        else node_go<T, 256, 2>(c, b, pl, check, partial, st, e0, e1);
    }
    return hipGetLastError();
}

template <typename T, int EPT, int UTIL>
static void fused_go(const Consts &c, const Bufs<T> &b, const PartLayout &pl, int parity, bool check, bool partial,
                     hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    constexpr int NWC = fused_waves<EPT, true>(), NWR = fused_waves<EPT, false>();
    constexpr size_t VW = EPT * 64 * sizeof(double);  // LDS bytes per wave for V (and T)
    const dim3 grid(c.n);
    if (check)
        MCF_LAUNCH((fused_kernel<T, EPT, UTIL, true, true>), grid, dim3(64 * NWC), 2 * NWC * VW, st, e0, e1,
                              0, c, b, pl, parity);
    else if (partial)
        MCF_LAUNCH((fused_kernel<T, EPT, UTIL, false, true>), grid, dim3(64 * NWR), NWR * VW, st, e0, e1,
                              0, c, b, pl, parity);
    else
        MCF_LAUNCH((fused_kernel<T, EPT, UTIL, false, false>), grid, dim3(64 * NWR), NWR * VW, st, e0, e1,
                              0, c, b, pl, parity);
}

template <typename T>
hipError_t launch_fused(const Consts &c, const Bufs<T> &b, const PartLayout &pl, EdgeShape, int parity, bool check,
                        bool partial, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
#define MCF_FUSED_CASE(E)                                                  \
    if (c.n <= 64 * E) {                                                   \
        if (c.utility == 0) fused_go<T, E, 0>(c, b, pl, parity, check, partial, st, e0, e1); \
        else if (c.utility == 1) fused_go<T, E, 1>(c, b, pl, parity, check, partial, st, e0, e1); \
        else fused_go<T, E, 2>(c, b, pl, parity, check, partial, st, e0, e1); \
        return hipGetLastError();                                          \
    }
    MCF_FUSED_CASE(1)
    MCF_FUSED_CASE(2)
    MCF_FUSED_CASE(4)
    MCF_FUSED_CASE(8)
#undef MCF_FUSED_CASE
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_residual(const Consts &c, const Bufs<T> &b, const PartLayout &pl, EdgeShape, hipStream_t st)
{
    hipLaunchKernelGGL(residual_kernel<T>, dim3(xcd_grid(c.nrp)), dim3(64 * RES_EDGES), 0, st, c, b, pl);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_control(const Consts &c, const Bufs<T> &b, const PartLayout &pl, bool check, bool adapt,
                          long long k_inc, hipStream_t st)
{
    // the longest segment the control reads (dF and dY only without a check)
    const long long most = check ? std::max(std::max((long long)c.nep, (long long)c.nnp), (long long)c.nrp)
                                 : std::max((long long)c.nep, (long long)c.nnp);
    const int split = most > CTRL_SPLIT_MIN ? 1 : 0;
    if (split)
        hipLaunchKernelGGL(control_split_kernel<T>, dim3(CTRL_GROUPS), dim3(CTRL_BLOCK), 0, st, c, b, pl,
                           check ? 1 : 0);
    hipLaunchKernelGGL(control_kernel<T>, dim3(1), dim3(CTRL_BLOCK), 0, st, c, b, pl, check ? 1 : 0, adapt ? 1 : 0,
                       k_inc, split);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_p_from_f(const Consts &c, const Bufs<T> &b, hipStream_t st)
{
    hipLaunchKernelGGL((p_from_f_kernel<T, 256>), dim3((c.n + 255) / 256, c.n), dim3(256), 0, st, c, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_poison(const Bufs<T> &b, int which, long long offset, hipStream_t st)
{
    hipLaunchKernelGGL(poison_kernel<T>, dim3(1), dim3(1), 0, st, b, which, offset);
    return hipGetLastError();
}

// Pool shapes compiled per iterate size: waves per node workgroup.
bool pool_waves_valid(int waves, int bytes)
{
    return waves == 8 || (bytes == 4 && (waves == 4 || waves == 2 || waves == 1));
}

// Measured pool shapes (written by tune.py), by the largest n a pool admits.
struct TunedPool {
    int bytes, n_max, waves, org;
};
#include "tuned_pool.inc"

int pool_org_for(int n, int bytes)
{
    for (const TunedPool &t : TUNED_POOL)
        if (t.bytes == bytes && n <= t.n_max) return t.org == 1 ? 1 : 0;
    return 0;
}

PoolShape pool_shape_for(int n_max, int bytes)
{
    PoolShape sh{8, 0, 0, n_max <= 64 ? 1 : n_max <= 128 ? 2 : n_max <= 256 ? 4 : 8, 0, 0};
    for (const TunedPool &t : TUNED_POOL)
        if (t.bytes == bytes && n_max <= t.n_max) {
            if (pool_waves_valid(t.waves, bytes)) sh.waves = t.waves;
            break;
        }
    return sh;
}

template <typename T, int NWV>
static void pool_fused_go(const SlotDesc<T> *slots, const int2 *work, const PoolState *ps, PoolShape sh, int it,
                          bool check, hipStream_t st)
{
    const size_t lds = (check ? 2 : 1) * NWV * sh.max_ept * 64 * sizeof(double);
    if (check)
        hipLaunchKernelGGL((pool_fused_kernel<T, NWV, true>), dim3(sh.grid), dim3(64 * NWV), lds, st, slots, work,
                           ps, it);
    else
        hipLaunchKernelGGL((pool_fused_kernel<T, NWV, false>), dim3(sh.grid), dim3(64 * NWV), lds, st, slots, work,
                           ps, it);
}

// sh.grid and sh.res_grid bound the item counts the pool state holds
template <typename T>
hipError_t launch_pool_iteration(const SlotDesc<T> *slots, const int2 *work, const int2 *ework, const int2 *nwork,
                                 const int *res_off, const PoolState *ps, int nslots, PoolShape sh, int it, bool check,
                                 bool control, hipStream_t st)
{
    if (!pool_waves_valid(sh.waves, sizeof(T))) return hipErrorInvalidValue;
    if (sh.edge_grid > 0) {  // two-phase slots: edge items (independent of the fused items)
        if (check)
            hipLaunchKernelGGL((pool_edge_kernel<T, true>), dim3(sh.edge_grid), dim3(64 * EDGE_PAR_WAVES), 0, st,
                               slots, ework, ps, it);
        else
            hipLaunchKernelGGL((pool_edge_kernel<T, false>), dim3(sh.edge_grid), dim3(64 * EDGE_PAR_WAVES), 0, st,
                               slots, ework, ps, it);
    }
    if (sh.grid < 1) {
        // no fused slots
    } else if (sh.waves == 8) pool_fused_go<T, 8>(slots, work, ps, sh, it, check, st);
    else if constexpr (sizeof(T) == 4) {
        if (sh.waves == 4) pool_fused_go<T, 4>(slots, work, ps, sh, it, check, st);
        else if (sh.waves == 2) pool_fused_go<T, 2>(slots, work, ps, sh, it, check, st);
        else pool_fused_go<T, 1>(slots, work, ps, sh, it, check, st);
    }
    if (sh.node_grid > 0) {  // two-phase slots: node items, after their edge items
        if (check)
            hipLaunchKernelGGL((pool_node_kernel<T, true>), dim3(sh.node_grid), dim3(64 * POOL_NODE_WAVES), 0, st,
                               slots, nwork, ps, it);
        else
            hipLaunchKernelGGL((pool_node_kernel<T, false>), dim3(sh.node_grid), dim3(64 * POOL_NODE_WAVES), 0, st,
                               slots, nwork, ps, it);
    }
    if (check && sh.res_grid > 0)
        hipLaunchKernelGGL(pool_residual_kernel<T>, dim3(sh.res_grid), dim3(64 * RES_EDGES), 0, st, slots, res_off, ps,
                           nslots, it);
    if (control)
        hipLaunchKernelGGL(pool_control_kernel<T>, dim3(nslots), dim3(CTRL_BLOCK), 0, st, slots, ps, it, check ? 1 : 0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pool_gather(const SlotDesc<T> *slots, int nslots, DevScalars *out, PoolState *ps, int iters,
                              hipStream_t st)
{
    hipLaunchKernelGGL(pool_gather_kernel<T>, dim3((nslots + 63) / 64), dim3(64), 0, st, slots, nslots, out, ps,
                       iters);
    return hipGetLastError();
}

#define MCF_INSTANTIATE(T)                                                                                      \
    template hipError_t launch_init<T>(const Consts &, const Bufs<T> &, double, hipStream_t);                   \
    template hipError_t launch_edge<T>(const Consts &, const Bufs<T> &, const PartLayout &, EdgeShape, bool,     \
                                       bool, hipStream_t, hipEvent_t, hipEvent_t);                              \
    template hipError_t launch_node<T>(const Consts &, const Bufs<T> &, const PartLayout &, bool, bool,          \
                                       hipStream_t, hipEvent_t, hipEvent_t);                                    \
    template hipError_t launch_fused<T>(const Consts &, const Bufs<T> &, const PartLayout &, EdgeShape, int, bool, \
                                        bool, hipStream_t, hipEvent_t, hipEvent_t);                             \
    template hipError_t launch_residual<T>(const Consts &, const Bufs<T> &, const PartLayout &, EdgeShape,       \
                                           hipStream_t);                                                        \
    template hipError_t launch_control<T>(const Consts &, const Bufs<T> &, const PartLayout &, bool, bool,       \
                                          long long, hipStream_t);                                              \
    template hipError_t launch_poison<T>(const Bufs<T> &, int, long long, hipStream_t);                      \
    template hipError_t launch_p_from_f<T>(const Consts &, const Bufs<T> &, hipStream_t);                    \
    template hipError_t launch_pool_iteration<T>(const SlotDesc<T> *, const int2 *, const int2 *, const int2 *,     \
                                                 const int *, const PoolState *, int, PoolShape, int, bool, bool, \
                                                 hipStream_t);                                                \
    template hipError_t launch_pool_gather<T>(const SlotDesc<T> *, int, DevScalars *, PoolState *, int, hipStream_t);

MCF_INSTANTIATE(float)
MCF_INSTANTIATE(double)

}  // namespace mcf

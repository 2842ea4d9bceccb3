// libmcf device kernels for gfx950 (CDNA4, wave64).
//
// One PDHG iteration of Algorithm 2.1 (eq. (e-pdhg-step)) is three launches:
//   edge phase  : per edge column l (destination-major, contiguous n-vector):
//                 q = F[:,l] + alpha (Y[:,head] - Y[:,tail]); Fhat = (q - mu)_+ (the
//                 projection of Section 2.3, mu from an exact active-set search);
//                 Fbar = 2 Fhat - F; F <- rho Fhat + (1 - rho) F; ||dF||^2 partial.
//   node phase  : per node column j: V = Fbar A^T as a deterministic gather over the
//                 in-edge and out-edge lists; Yhat = prox(Y - beta V) off the diagonal,
//                 0 on it (Section 2.3); Y <- rho Yhat + (1 - rho) Y; ||dY||^2 partial.
//   control     : FP64 fixed-order reduction of the partials, the adaptive primal
//                 weight (e-primal_weight), the stop flag.
// On check iterations the edge and node phases also produce Fhat, D = Fhat - Q,
// T = -Fhat A^T and U' = u'(T), and a residual pass forms ||G||^2 and <G, D> for
// r(Q) of (e-res).  No atomics anywhere: every sum has a fixed order.
#include <math.h>

#include "mcf_internal.h"

namespace mcf {

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Block-wide sums of x and y, returned identically to every thread.  The wave
// partials are combined in wave order, so the result is deterministic.
template <int BLOCK>
__device__ __forceinline__ void block_sum2(double &x, double &y, double *lds)
{
    x = wave_sum(x);
    y = wave_sum(y);
    if constexpr (BLOCK > 64) {
        constexpr int NW = BLOCK / 64;
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
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

template <int BLOCK>
__device__ __forceinline__ double block_max(double x, double *lds)
{
    x = wave_max(x);
    if constexpr (BLOCK > 64) {
        constexpr int NW = BLOCK / 64;
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
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
// Section 1.1: u(s) = w log s (log) or w s^gamma (power); u' for U' = u'(T);
// the conjugate (-u)^*(y) and the traffic s(y) maximizing y s + u(s), both for y < 0.
template <int UTIL>
__device__ __forceinline__ double util_u(double s, double w, double g)
{
    return UTIL == 0 ? w * log(s) : w * pow(s, g);
}
template <int UTIL>
__device__ __forceinline__ double util_du(double s, double w, double g)
{
    return UTIL == 0 ? w / s : w * g * pow(s, g - 1.0);
}
template <int UTIL>
__device__ __forceinline__ double util_conj(double y, double w, double g)
{
    if (UTIL == 0) return -w + w * log(w) - w * log(-y);
    return (1.0 / g - 1.0) * pow(w * g, 1.0 / (1.0 - g)) * pow(-y, -g / (1.0 - g));
}
template <int UTIL>
__device__ __forceinline__ double util_traffic(double y, double w, double g)
{
    return UTIL == 0 ? w / (-y) : pow(w * g / (-y), 1.0 / (1.0 - g));
}

// Dual proximal operator prox_{beta (-u)^*}(y) of Section 2.3.
//   log:   (y - sqrt(y^2 + 4 beta w)) / 2, in the cancellation-free form for y > 0;
//   power: z = -t with t the positive root of t^{c1+2} + y t^{c1+1} = c1 c2.  On
//          t >= max(-y, 0) that polynomial is increasing and convex, so Newton's
//          method started right of the root, at max(-y,0) + (c1 c2)^{1/(c1+2)},
//          decreases monotonically onto it; it stops when a step no longer decreases t.
template <int UTIL>
__device__ __forceinline__ double prox_dual(double y, double beta, double w, double g, double c1)
{
    if (UTIL == 0) {
        const double s = sqrt(y * y + 4.0 * beta * w);
        return y <= 0.0 ? 0.5 * (y - s) : -2.0 * beta * w / (y + s);
    }
    const double a = y < 0.0 ? -y : 0.0;
    if (c1 == 1.0) {  // gamma = 1/2: t^3 + y t^2 - beta w^2 / 4 = 0
        const double k = beta * w * w * 0.25;
        double t = a + cbrt(k);
        for (int it = 0; it < 200; ++it) {
            const double h = t * t * (t + y) - k;
            const double hp = t * (3.0 * t + 2.0 * y);
            const double tn = t - h / hp;
            if (!(tn < t)) break;
            t = tn > a ? tn : a;
        }
        return -t;
    }
    const double k = c1 * beta * (1.0 / g - 1.0) * pow(w * g, 1.0 / (1.0 - g));
    double t = a + pow(k, 1.0 / (c1 + 2.0));
    for (int it = 0; it < 200; ++it) {
        const double tp = pow(t, c1);
        const double h = tp * t * (t + y) - k;
        const double hp = tp * ((c1 + 2.0) * t + (c1 + 1.0) * y);
        const double tn = t - h / hp;
        if (!(tn < t)) break;
        t = tn > a ? tn : a;
    }
    return -t;
}

// ------------------------------------------------------------------- init
template <typename T>
__global__ void init_kernel(Consts c, Bufs<T> b, double omega0)
{
    const long long nm = c.ld * (long long)c.m, nn = c.ld * (long long)c.n;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < nm; x += stride) {
        b.F[x] = T(0);
        b.Fhat[x] = T(0);
    }
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < nn; x += stride) {
        const long long j = x / c.ld, i = x - j * c.ld;
        // Section 2.5 initialization: Y^0 = I - 1 1^T (0 on the diagonal, -1 off it); padding stays 0.
        b.Y[x] = (i < c.n && i != j) ? T(-1) : T(0);
        b.That[x] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
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
// One workgroup per edge column; each thread keeps EPT entries of F[:,l] and q in
// registers.  mu (Section 2.3, Section 2.6): if sum (q)_+ <= c the projection is (q)_+;
// otherwise the active set S = {q_i > mu} and mu = (sum_S q - c)/|S| are iterated from
// S = {q > 0}.  mu only grows and S only shrinks, so the loop ends when |S| stops
// shrinking; the final mu is the exact value (sum_S q - c)/|S| on the support S.
template <typename T, int BLOCK, int EPT, bool CHECK>
__global__ __launch_bounds__(BLOCK) void edge_kernel(Consts c, Bufs<T> b, PartLayout pl)
{
    __shared__ double lds[2 * (BLOCK / 64)];
    if (b.sc->stop) return;
    const int e = blockIdx.x;
    const int n = c.n;
    const long long ld = c.ld;
    const T ta = (T)b.sc->alpha;
    const T *yh = b.Y + (long long)b.head[e] * ld;
    const T *yt = b.Y + (long long)b.tail[e] * ld;
    T *f = b.F + (long long)e * ld;
    T fo[EPT], q[EPT];
    double s = 0.0, cnt = 0.0;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int i = threadIdx.x + j * BLOCK;
        if (i < n) {
            fo[j] = f[i];
            q[j] = fo[j] + ta * (yh[i] - yt[i]);
            if (q[j] > T(0)) {
                s += (double)q[j];
                cnt += 1.0;
            }
        } else {
            fo[j] = T(0);
            q[j] = T(-1);  // never in the support
        }
    }
    block_sum2<BLOCK>(s, cnt, lds);
    const double cap = b.cap[e];
    double mu = 0.0;
    if (s > cap) {
        mu = (s - cap) / cnt;
        double prev = cnt;
        for (int pass = 0; pass <= n; ++pass) {
            s = 0.0;
            cnt = 0.0;
#pragma unroll
            for (int j = 0; j < EPT; ++j)
                if ((double)q[j] > mu) {
                    s += (double)q[j];
                    cnt += 1.0;
                }
            block_sum2<BLOCK>(s, cnt, lds);
            if (cnt >= prev) break;
            mu = (s - cap) / cnt;
            prev = cnt;
        }
    }
    T *fb = b.Fbar + (long long)e * ld;
    const double rho = c.rho, omr = 1.0 - c.rho;
    double dsum = 0.0, esum = 0.0, gmax = -INFINITY;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int i = threadIdx.x + j * BLOCK;
        if (i < n) {
            const double fod = (double)fo[j];
            const double fh = fmax((double)q[j] - mu, 0.0);
            const T fn = (T)(rho * fh + omr * fod);
            f[i] = fn;
            fb[i] = (T)(2.0 * fh - fod);
            const double d = (double)fn - fod;
            dsum += d * d;
            if (CHECK) {
                b.Fhat[(long long)e * ld + i] = (T)fh;
                const T dd = (T)(fh - (double)q[j]);
                b.D[(long long)e * ld + i] = dd;
                esum += (double)dd * (double)dd;
                gmax = fmax(gmax, (double)(yh[i] - yt[i]));
            }
        }
    }
    block_sum2<BLOCK>(dsum, esum, lds);
    if (CHECK) gmax = block_max<BLOCK>(gmax, lds);
    if (threadIdx.x == 0) {
        b.part[pl.dF + e] = dsum;
        if (CHECK) {
            b.part[pl.e + e] = esum;
            b.part[pl.sup + e] = cap * fmax(gmax, 0.0);  // c_l (max_i (Y A)_il)_+
        }
    }
}

// -------------------------------------------------------------- node phase
// Grid (ceil(n/NODE_BLOCK), n): thread (x, j) owns entry i of node column j.
// V_ij = sum_{l in in(j)} Fbar_il - sum_{l in out(j)} Fbar_il, in CSR order, FP64.
template <typename T, int UTIL, bool CHECK>
__global__ __launch_bounds__(NODE_BLOCK) void node_kernel(Consts c, Bufs<T> b, PartLayout pl)
{
    __shared__ double lds[2 * (NODE_BLOCK / 64)];
    if (b.sc->stop) return;
    const int j = blockIdx.y;
    const int i = blockIdx.x * NODE_BLOCK + threadIdx.x;
    const int blk = blockIdx.y * gridDim.x + blockIdx.x;
    const long long ld = c.ld;
    const double beta = b.sc->beta, g = c.gamma;
    double dy2 = 0.0, p = 0.0, conj = 0.0, rnum = 0.0, rden = 0.0, nonpos = 0.0, yinf = 0.0;
    if (i < c.n) {
        const int i0 = b.in_off[j], i1 = b.in_off[j + 1], o0 = b.out_off[j], o1 = b.out_off[j + 1];
        double v = 0.0;
        for (int k = i0; k < i1; ++k) v += (double)b.Fbar[(long long)b.in_edge[k] * ld + i];
        for (int e = o0; e < o1; ++e) v -= (double)b.Fbar[(long long)e * ld + i];
        const long long x = (long long)j * ld + i;
        const double y = (double)b.Y[x];
        const double w = (double)b.W[x];
        const double yhat = (i != j) ? prox_dual<UTIL>(y - beta * v, beta, w, g, c.c1) : 0.0;
        const T yn = (T)(c.rho * yhat + (1.0 - c.rho) * y);
        b.Y[x] = yn;
        const double d = (double)yn - y;
        dy2 = d * d;
        if (CHECK) {
            // T = -Fhat A^T, U' = u'(T), and the pieces of p, d and rel_primal (with Y^k = y).
            double t = 0.0;
            for (int k = i0; k < i1; ++k) t -= (double)b.Fhat[(long long)b.in_edge[k] * ld + i];
            for (int e = o0; e < o1; ++e) t += (double)b.Fhat[(long long)e * ld + i];
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
    double zero = 0.0;
    block_sum2<NODE_BLOCK>(dy2, zero, lds);
    if (CHECK) {
        block_sum2<NODE_BLOCK>(p, conj, lds);
        block_sum2<NODE_BLOCK>(rnum, rden, lds);
        block_sum2<NODE_BLOCK>(nonpos, yinf, lds);
    }
    if (threadIdx.x == 0) {
        b.part[pl.dY + blk] = dy2;
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

// ---------------------------------------------------------- residual pass
// Per edge: G[:,l] = U'[:,head] - U'[:,tail]; partials ||G_l||^2 and <G_l, D_l>.
template <typename T, int BLOCK>
__global__ __launch_bounds__(BLOCK) void residual_kernel(Consts c, Bufs<T> b, PartLayout pl)
{
    __shared__ double lds[2 * (BLOCK / 64)];
    if (b.sc->stop) return;
    const int e = blockIdx.x;
    const long long ld = c.ld;
    const double *uh = b.Up + (long long)b.head[e] * ld;
    const double *ut = b.Up + (long long)b.tail[e] * ld;
    const T *d = b.D + (long long)e * ld;
    double a = 0.0, bb = 0.0;
    for (int i = threadIdx.x; i < c.n; i += BLOCK) {
        const double gg = uh[i] - ut[i];
        a += gg * gg;
        bb += gg * (double)d[i];
    }
    block_sum2<BLOCK>(a, bb, lds);
    if (threadIdx.x == 0) {
        b.part[pl.a + e] = a;
        b.part[pl.b + e] = bb;
    }
}

// ----------------------------------------------------------------- control
constexpr int CTRL_BLOCK = 256;

__device__ double seg_sum(const double *p, long long len, double *lds)
{
    double s = 0.0;
    for (long long x = threadIdx.x; x < len; x += CTRL_BLOCK) s += p[x];
    double z = 0.0;
    block_sum2<CTRL_BLOCK>(s, z, lds);
    return s;
}

template <typename T>
__global__ __launch_bounds__(CTRL_BLOCK) void control_kernel(Consts c, Bufs<T> b, PartLayout pl, int check)
{
    __shared__ double lds[2 * (CTRL_BLOCK / 64)];
    DevScalars *sc = b.sc;
    if (sc->stop) return;
    const double *P = b.part;
    const double dF2 = seg_sum(P + pl.dF, c.m, lds);
    const double dY2 = seg_sum(P + pl.dY, c.nblk_node, lds);
    double e = 0, sup = 0, a = 0, bb = 0, psum = 0, conj = 0, rnum = 0, rden = 0, nonpos = 0, yinf = 0;
    if (check) {
        e = seg_sum(P + pl.e, c.m, lds);
        sup = seg_sum(P + pl.sup, c.m, lds);
        a = seg_sum(P + pl.a, c.m, lds);
        bb = seg_sum(P + pl.b, c.m, lds);
        psum = seg_sum(P + pl.p, c.nblk_node, lds);
        conj = seg_sum(P + pl.conj, c.nblk_node, lds);
        rnum = seg_sum(P + pl.rnum, c.nblk_node, lds);
        rden = seg_sum(P + pl.rden, c.nblk_node, lds);
        nonpos = seg_sum(P + pl.nonpos, c.nblk_node, lds);
        yinf = seg_sum(P + pl.yinf, c.nblk_node, lds);
    }
    if (threadIdx.x != 0) return;
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
    const long long k = sc->k;
    const bool bad = !isfinite(dF) || !isfinite(dY);
    // Algorithm 2.1 step 3, (e-primal_weight)
    if (!bad && c.k_adapt > 0 && k % c.k_adapt == 0 && dF > c.tau && dY > c.tau) {
        const double om = pow(dY / dF, c.theta) * pow(sc->omega, 1.0 - c.theta);
        sc->omega = om;
        sc->alpha = sc->eta / om;
        sc->beta = sc->eta * om;
    }
    sc->k = k + 1;
    if (bad) {
        sc->state = 3;
        sc->stop = 1;
    } else if (converged && sc->stop_enabled) {
        sc->state = 1;
        sc->stop = 1;
    }
}

template <typename T>
__global__ void poison_kernel(Bufs<T> b, int which, long long off)
{
    if (which == 0) b.F[off] = (T)NAN;
    else b.Y[off] = (T)NAN;
}

// ---------------------------------------------------------------- launchers
EdgeShape edge_shape_for(int n)
{
    if (n <= 64) return {64, 1};
    if (n <= 128) return {64, 2};
    if (n <= 256) return {64, 4};
    if (n <= 512) return {128, 4};
    if (n <= 1024) return {256, 4};
    if (n <= 2048) return {256, 8};
    if (n <= 4096) return {512, 8};
    if (n <= 8192) return {512, 16};
    return {1024, 16};
}

template <typename T>
hipError_t launch_init(const Consts &c, const Bufs<T> &b, double omega0, hipStream_t st)
{
    hipLaunchKernelGGL(init_kernel<T>, dim3(1024), dim3(256), 0, st, c, b, omega0);
    return hipGetLastError();
}

template <typename T, int BLOCK, int EPT>
static void edge_go(const Consts &c, const Bufs<T> &b, const PartLayout &pl, bool check, hipStream_t st)
{
    if (check)
        hipLaunchKernelGGL((edge_kernel<T, BLOCK, EPT, true>), dim3(c.m), dim3(BLOCK), 0, st, c, b, pl);
    else
        hipLaunchKernelGGL((edge_kernel<T, BLOCK, EPT, false>), dim3(c.m), dim3(BLOCK), 0, st, c, b, pl);
}

template <typename T>
hipError_t launch_edge(const Consts &c, const Bufs<T> &b, const PartLayout &pl, EdgeShape sh, bool check,
                       hipStream_t st)
{
#define MCF_EDGE_CASE(B, E) \
    if (sh.block == B && sh.ept == E) { edge_go<T, B, E>(c, b, pl, check, st); return hipGetLastError(); }
    MCF_EDGE_CASE(64, 1)
    MCF_EDGE_CASE(64, 2)
    MCF_EDGE_CASE(64, 4)
    MCF_EDGE_CASE(128, 4)
    MCF_EDGE_CASE(256, 4)
    MCF_EDGE_CASE(256, 8)
    MCF_EDGE_CASE(512, 8)
    MCF_EDGE_CASE(512, 16)
    MCF_EDGE_CASE(1024, 16)
#undef MCF_EDGE_CASE
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_node(const Consts &c, const Bufs<T> &b, const PartLayout &pl, bool check, hipStream_t st)
{
    const dim3 grid((c.n + NODE_BLOCK - 1) / NODE_BLOCK, c.n);
    if (c.utility == 0) {
        if (check) hipLaunchKernelGGL((node_kernel<T, 0, true>), grid, dim3(NODE_BLOCK), 0, st, c, b, pl);
        else hipLaunchKernelGGL((node_kernel<T, 0, false>), grid, dim3(NODE_BLOCK), 0, st, c, b, pl);
    } else {
        if (check) hipLaunchKernelGGL((node_kernel<T, 1, true>), grid, dim3(NODE_BLOCK), 0, st, c, b, pl);
        else hipLaunchKernelGGL((node_kernel<T, 1, false>), grid, dim3(NODE_BLOCK), 0, st, c, b, pl);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_residual(const Consts &c, const Bufs<T> &b, const PartLayout &pl, EdgeShape sh, hipStream_t st)
{
    if (sh.block <= 64) hipLaunchKernelGGL((residual_kernel<T, 64>), dim3(c.m), dim3(64), 0, st, c, b, pl);
    else hipLaunchKernelGGL((residual_kernel<T, 256>), dim3(c.m), dim3(256), 0, st, c, b, pl);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_control(const Consts &c, const Bufs<T> &b, const PartLayout &pl, bool check, hipStream_t st)
{
    hipLaunchKernelGGL(control_kernel<T>, dim3(1), dim3(CTRL_BLOCK), 0, st, c, b, pl, check ? 1 : 0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_poison(const Bufs<T> &b, int which, long long offset, hipStream_t st)
{
    hipLaunchKernelGGL(poison_kernel<T>, dim3(1), dim3(1), 0, st, b, which, offset);
    return hipGetLastError();
}

#define MCF_INSTANTIATE(T)                                                                                  \
    template hipError_t launch_init<T>(const Consts &, const Bufs<T> &, double, hipStream_t);               \
    template hipError_t launch_edge<T>(const Consts &, const Bufs<T> &, const PartLayout &, EdgeShape, bool, \
                                       hipStream_t);                                                        \
    template hipError_t launch_node<T>(const Consts &, const Bufs<T> &, const PartLayout &, bool, hipStream_t); \
    template hipError_t launch_residual<T>(const Consts &, const Bufs<T> &, const PartLayout &, EdgeShape,   \
                                           hipStream_t);                                                    \
    template hipError_t launch_control<T>(const Consts &, const Bufs<T> &, const PartLayout &, bool,         \
                                          hipStream_t);                                                     \
    template hipError_t launch_poison<T>(const Bufs<T> &, int, long long, hipStream_t);

MCF_INSTANTIATE(float)
MCF_INSTANTIATE(double)

}  // namespace mcf

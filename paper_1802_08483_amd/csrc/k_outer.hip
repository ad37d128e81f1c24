// Belief propagation for the outer code of iterative decoding (Sec. II-A:
// serial concatenation; the inner decoder's priors from the outer decoder's
// extrinsic output).  Linear code over GF(q), q = 2^p <= 64, sum-product on
// its factor graph, flooding schedule.
//
// Check update, one wave per (check c, frame), lane = field element: the
// message to symbol j is the distribution of s = sum_{k != j} H[c][k] x_k
// evaluated at H[c][j] a.  Distributions of sums under XOR multiply under
// the Walsh-Hadamard transform, so each incoming message v(k->c) is
// gathered through the coefficient (w_k(b) = v(k->c)(H[c][k]^-1 b)),
// transformed across the lanes (log2 q butterfly stages of lane shuffles),
// the transforms of all but one edge multiplied (suffix products in LDS, a
// running prefix in registers), transformed back (the transform is its own
// inverse up to 1/q) and read at H[c][j] a with a lane permutation.
// Rounding can leave tiny negative values: they are clamped to 0 before
// the message is normalised.
//
// Symbol update, one wave per (symbol j, frame), lane = field element:
// v(j->c)(a) proportional to L_j(a) prod_{c' != c} u(c'->j)(a); after the
// last iteration extrinsic prod_c u(c->j)(a) and posterior L_j(a) prod_c
// u(c->j)(a).  L_j is the channel row divided by its sum.  Every message
// is normalised to sum 1; a vector summing to 0 becomes uniform.
#include "device_common.h"

namespace mapdec {

namespace {

template <typename T>
__device__ __forceinline__ T wave_total(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// unnormalised Walsh-Hadamard transform over the first q lanes
template <typename T>
__device__ __forceinline__ T wht(T v, int lane, int q) {
    for (int bit = 1; bit < q; bit <<= 1) {
        const T o = __shfl_xor(v, bit, 64);
        v = (lane & bit) ? (o - v) : (v + o);
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T normalised(T v, bool live, int q) {
    const T s = wave_total(live ? v : T(0));
    return s > T(0) ? v / s : T(1) / T(q);
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(64) void k_outer_check(OuterDev c, const T *__restrict__ v2c,
                                                    T *__restrict__ c2v) {
    const int row = blockIdx.x, f = blockIdx.y, a = threadIdx.x, q = c.q;
    const bool live = a < q;
    const int e0 = c.row_ptr[row], d = c.row_ptr[row + 1] - e0;
    const size_t fo = (size_t)f * c.E * q;
    __shared__ T W[kOuterMaxDeg][64];        // transforms of the incoming messages
    __shared__ T S[kOuterMaxDeg + 1][64];    // suffix products of W
    for (int k = 0; k < d; ++k) {
        const int e = e0 + k;
        const int hi = c.inv[c.coef[e]];
        const int x = live ? c.mul[hi * q + a] : 0;
        const T w = live ? v2c[fo + (size_t)e * q + x] : T(0);
        W[k][a] = wht(w, a, q);
    }
    S[d][a] = T(1);
    for (int k = d - 1; k >= 0; --k) S[k][a] = W[k][a] * S[k + 1][a];
    T pre = T(1);
    for (int t = 0; t < d; ++t) {
        const int e = e0 + t;
        T s = wht(pre * S[t + 1][a], a, q) / T(q);   // distribution of the other terms
        pre *= W[t][a];
        const int src = live ? c.mul[c.coef[e] * q + a] : 0;
        T u = __shfl(s, src, 64);
        u = u > T(0) ? u : T(0);
        u = normalised(u, live, q);
        if (live) c2v[fo + (size_t)e * q + a] = u;
    }
}

// mode 0: first pass (v = L on every edge); 1: update v from the checks;
// 2: last pass (extrinsic and posterior out)
template <typename T>
__global__ __launch_bounds__(64) void k_outer_var(OuterDev c, const T *__restrict__ chan,
                                                  const T *__restrict__ c2v, T *__restrict__ v2c,
                                                  T *__restrict__ extr, T *__restrict__ post,
                                                  int mode) {
    const int j = blockIdx.x, f = blockIdx.y, a = threadIdx.x, q = c.q;
    const bool live = a < q;
    const size_t fo = (size_t)f * c.E * q;
    const size_t ro = ((size_t)f * c.N + j) * q;
    const int k0 = c.var_ptr[j], dv = c.var_ptr[j + 1] - k0;
    const T L = normalised(live ? chan[ro + a] : T(0), live, q);
    if (mode == 0) {
        for (int k = 0; k < dv; ++k)
            if (live) v2c[fo + (size_t)c.var_edge[k0 + k] * q + a] = L;
        return;
    }
    __shared__ T U[kOuterMaxDeg][64];
    for (int k = 0; k < dv; ++k)
        U[k][a] = live ? c2v[fo + (size_t)c.var_edge[k0 + k] * q + a] : T(0);
    if (mode == 1) {
        for (int k = 0; k < dv; ++k) {
            T p = L;
            for (int k2 = 0; k2 < dv; ++k2)
                if (k2 != k) p *= U[k2][a];
            p = normalised(p, live, q);
            if (live) v2c[fo + (size_t)c.var_edge[k0 + k] * q + a] = p;
        }
        return;
    }
    T ext = T(1);
    for (int k = 0; k < dv; ++k) ext *= U[k][a];
    const T E = normalised(ext, live, q);
    const T Q = normalised(L * ext, live, q);
    if (live) {
        extr[ro + a] = E;
        if (post) post[ro + a] = Q;
    }
}

template <typename T>
static hipError_t outer_run(const OuterDev &c, int nframes, const T *chan, T *extr, T *post,
                            int iters, T *v2c, T *c2v, hipStream_t st) {
    const dim3 gv(c.N, nframes), gc(c.m, nframes);
    if (c.N > 0) hipLaunchKernelGGL(k_outer_var<T>, gv, dim3(64), 0, st, c, chan, c2v, v2c, extr,
                                    post, 0);
    for (int it = 1; it <= iters; ++it) {
        if (c.m > 0) hipLaunchKernelGGL(k_outer_check<T>, gc, dim3(64), 0, st, c, v2c, c2v);
        if (c.N > 0)
            hipLaunchKernelGGL(k_outer_var<T>, gv, dim3(64), 0, st, c, chan, c2v, v2c, extr,
                               post, it == iters ? 2 : 1);
    }
    return hipGetLastError();
}

hipError_t launch_outer(int fp64, const OuterDev &c, int nframes, const void *chan, void *extr,
                        void *post, int iters, void *v2c, void *c2v, hipStream_t st) {
    if (nframes == 0) return hipSuccess;
    if (fp64)
        return outer_run<double>(c, nframes, (const double *)chan, (double *)extr, (double *)post,
                                 iters, (double *)v2c, (double *)c2v, st);
    return outer_run<float>(c, nframes, (const float *)chan, (float *)extr, (float *)post, iters,
                            (float *)v2c, (float *)c2v, st);
}

}  // namespace mapdec

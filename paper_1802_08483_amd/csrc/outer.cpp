// Host side of the outer code of iterative decoding (Sec. II-A): validation,
// the code's device tables, workspace and launches.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "kernels.h"
#include "mapdec.h"
#include "mapdec_internal.h"

using namespace mapdec;

struct mapdec_outer {
    int q = 0, N = 0, m = 0, E = 0;
    int device = 0;
    void *buf = nullptr;    // one device allocation holding every table
    OuterDev d{};
};

namespace {

// Primitive polynomials of GF(2^p), bit k = coefficient of z^k.
constexpr unsigned kPrimitive[7] = {0, 0x3, 0x7, 0xB, 0x13, 0x25, 0x43};

int field_bits(int q) {
    for (int p = 1; p <= 6; ++p)
        if (q == (1 << p)) return p;
    return 0;
}

// Multiplication table of GF(2^p) from the powers of z: z^k by repeated
// multiplication by z (shift, and reduction when degree p appears).
void field_tables(int p, std::vector<uint8_t> &mul, std::vector<uint8_t> &inv) {
    const int q = 1 << p;
    std::vector<int> pw(q - 1), lg(q, -1);
    unsigned e = 1;
    for (int k = 0; k < q - 1; ++k) {
        pw[k] = (int)e;
        lg[e] = k;
        e <<= 1;
        if (e & (unsigned)q) e ^= kPrimitive[p];
    }
    mul.assign((size_t)q * q, 0);
    inv.assign(q, 0);
    for (int a = 1; a < q; ++a) {
        for (int b = 1; b < q; ++b) mul[(size_t)a * q + b] = (uint8_t)pw[(lg[a] + lg[b]) % (q - 1)];
        inv[a] = (uint8_t)pw[(q - 1 - lg[a]) % (q - 1)];
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

mapdec_outer *mapdec_outer_create(int q, int N, int m, const int32_t *row_ptr,
                                  const int32_t *col, const uint8_t *coef) {
    const int p = field_bits(q);
    if (!p || N < 1 || m < 0 || !row_ptr || row_ptr[0] != 0) {
        record_error(MAPDEC_EINVAL);
        return nullptr;
    }
    const int E = row_ptr[m];
    if (E < 0 || (E > 0 && (!col || !coef))) {
        record_error(MAPDEC_EINVAL);
        return nullptr;
    }
    std::vector<int> deg(N, 0), seen(N, -1);
    for (int r = 0; r < m; ++r) {
        if (row_ptr[r + 1] < row_ptr[r]) {
            record_error(MAPDEC_EINVAL);
            return nullptr;
        }
        if (row_ptr[r + 1] - row_ptr[r] > MAPDEC_OUTER_MAX_DEG) {
            record_error(MAPDEC_EUNSUPPORTED);
            return nullptr;
        }
        for (int e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
            if (col[e] < 0 || col[e] >= N || coef[e] == 0 || coef[e] >= q || seen[col[e]] == r) {
                record_error(MAPDEC_EINVAL);
                return nullptr;
            }
            seen[col[e]] = r;
            if (++deg[col[e]] > MAPDEC_OUTER_MAX_DEG) {
                record_error(MAPDEC_EUNSUPPORTED);
                return nullptr;
            }
        }
    }
    // edges of every symbol, in edge order
    std::vector<int> var_ptr(N + 1, 0), var_edge(E), fill(N, 0);
    for (int j = 0; j < N; ++j) var_ptr[j + 1] = var_ptr[j] + deg[j];
    for (int e = 0; e < E; ++e) var_edge[var_ptr[col[e]] + fill[col[e]]++] = e;
    std::vector<uint8_t> mul, inv;
    field_tables(p, mul, inv);

    mapdec_outer *c = new (std::nothrow) mapdec_outer;
    if (!c) {
        record_error(MAPDEC_ENOMEM);
        return nullptr;
    }
    c->q = q; c->N = N; c->m = m; c->E = E;
    // layout: row_ptr, col, var_ptr, var_edge (int32), coef, mul, inv (bytes)
    const size_t o_row = 0, o_col = align256(o_row + sizeof(int) * (m + 1));
    const size_t o_vp = align256(o_col + sizeof(int) * (size_t)E);
    const size_t o_ve = align256(o_vp + sizeof(int) * (size_t)(N + 1));
    const size_t o_coef = align256(o_ve + sizeof(int) * (size_t)E);
    const size_t o_mul = align256(o_coef + (size_t)E);
    const size_t o_inv = align256(o_mul + (size_t)q * q);
    const size_t bytes = align256(o_inv + (size_t)q);
    std::vector<unsigned char> host(bytes, 0);
    std::memcpy(host.data() + o_row, row_ptr, sizeof(int) * (m + 1));
    if (E) {
        std::memcpy(host.data() + o_col, col, sizeof(int) * (size_t)E);
        std::memcpy(host.data() + o_ve, var_edge.data(), sizeof(int) * (size_t)E);
        std::memcpy(host.data() + o_coef, coef, (size_t)E);
    }
    std::memcpy(host.data() + o_vp, var_ptr.data(), sizeof(int) * (size_t)(N + 1));
    std::memcpy(host.data() + o_mul, mul.data(), (size_t)q * q);
    std::memcpy(host.data() + o_inv, inv.data(), (size_t)q);
    if (hipGetDevice(&c->device) != hipSuccess || hipMalloc(&c->buf, bytes) != hipSuccess) {
        delete c;
        record_error(MAPDEC_EDEVICE);
        return nullptr;
    }
    if (hipMemcpy(c->buf, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(c->buf);
        delete c;
        record_error(MAPDEC_EDEVICE);
        return nullptr;
    }
    unsigned char *b = (unsigned char *)c->buf;
    c->d.q = q; c->d.N = N; c->d.m = m; c->d.E = E;
    c->d.row_ptr = (const int *)(b + o_row);
    c->d.col = (const int *)(b + o_col);
    c->d.var_ptr = (const int *)(b + o_vp);
    c->d.var_edge = (const int *)(b + o_ve);
    c->d.coef = b + o_coef;
    c->d.mul = b + o_mul;
    c->d.inv = b + o_inv;
    return c;
}

void mapdec_outer_destroy(mapdec_outer *c) {
    if (!c) return;
    if (c->buf) (void)hipFree(c->buf);
    delete c;
}

size_t mapdec_outer_workspace_size(const mapdec_outer *c, int nframes, int precision) {
    if (!c || nframes < 0 || (precision != MAPDEC_FP32 && precision != MAPDEC_FP64)) return 0;
    const size_t t = precision == MAPDEC_FP64 ? 8 : 4;
    // both message directions of every edge of every frame
    return 2 * align256((size_t)nframes * c->E * c->q * t) + 256;
}

int mapdec_outer_decode(const mapdec_outer *c, int nframes, const void *chan, void *extr,
                        void *post, int iters, void *ws, size_t ws_bytes, int precision,
                        void *stream) {
    if (!c || nframes < 0 || nframes > 65535 || iters < 1 ||
        (precision != MAPDEC_FP32 && precision != MAPDEC_FP64))
        return MAPDEC_EINVAL;
    if (nframes == 0) return MAPDEC_OK;
    if (!chan || !extr || !ws) return MAPDEC_EINVAL;
    if (ws_bytes < mapdec_outer_workspace_size(c, nframes, precision)) return MAPDEC_ESIZE;
    const size_t t = precision == MAPDEC_FP64 ? 8 : 4;
    unsigned char *w = (unsigned char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    void *v2c = w;
    void *c2v = w + align256((size_t)nframes * c->E * c->q * t);
    const hipError_t e = launch_outer(precision == MAPDEC_FP64, c->d, nframes, chan, extr, post,
                                      iters, v2c, c2v, (hipStream_t)stream);
    return e == hipSuccess ? MAPDEC_OK : MAPDEC_EDEVICE;
}

}  // extern "C"

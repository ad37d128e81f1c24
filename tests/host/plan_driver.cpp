// Drives libmapdec's host code (linked against plan_stub.cpp) through plan
// creation, runs, profiling, tuning and destruction on uneven and uniform
// batches; the stub aborts on any out-of-range table, unknown handle or
// launch not ordered after an earlier launch of one of its frames.
//   plan_driver <frames> <checkpoint_K> <flags> <mode: 0 uneven, 1 uniform, 2 general,
//                                                3 uniform frames of the long-frame code>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "mapdec.h"

void stub_set_workspace(void *p, size_t bytes, size_t alloc, int nframes);
long stub_launches();
long stub_waits();
int stub_live_objects();

int main(int argc, char **argv) {
    if (argc < 5) return 2;
    const int nf = atoi(argv[1]), K = atoi(argv[2]), flags = atoi(argv[3]);
    // mode: 0 uneven batch, 1 uniform batch, 2 uneven with general-scheme
    // frames, 3 uniform batch of 64 codewords of 12 bits (the MFMA APP)
    const int mode = atoi(argv[4]);
    const bool uniform = mode == 1 || mode == 3;
    std::mt19937 rng(1802);
    std::vector<mapdec_code *> codes;
    std::vector<mapdec_frame> fr(nf);
    static unsigned char dev[16];   // stands in for device buffers the stub never reads
    for (int f = 0; f < nf; ++f) {
        int q = 16, n = 10, N = 200, mn = 6;
        double p = 0.05;
        if (mode == 3) {
            q = 64;
            n = 12;
            N = 150;
            mn = 8;
            p = 0.1;
        }
        if (!uniform) {
            const int qs[3] = {2, 8, 16};
            q = qs[rng() % 3];
            const int nmin = q == 16 ? 5 : 4;
            n = nmin + (int)(rng() % (11 - nmin));
            N = 50 + (int)(rng() % 600);
            p = std::pow(10.0, -3.0 + 2.0 * (double)(rng() % 1000) / 1000.0);
            mn = 3 + (int)(rng() % 5);
        }
        int M = (int)std::ceil(6.0 * std::sqrt(n * N * p / (1.0 - p))) + 2;
        if (mode == 3) M = 85;
        if (M < mn) M = mn;
        std::vector<uint8_t> cb((size_t)q * n);
        for (int D = 0; D < q; ++D)
            for (int r = 0; r < n; ++r) cb[(size_t)D * n + r] = (uint8_t)((D >> (r % 5)) & 1);
        for (int D = 0; D < q; ++D)   // distinct: the low bits of D in the first 6 positions
            for (int r = 0; r < 6 && r < n; ++r) cb[(size_t)D * n + r] = (uint8_t)((D >> r) & 1);
        mapdec_code *c = nullptr;
        if (mode == 2 && f % 3 == 0) {
            // the general scheme: a codebook per symbol (the same words,
            // rotated per position) and asymmetric limits
            std::vector<uint8_t> cbs((size_t)N * q * n);
            for (int i = 0; i < N; ++i)
                for (int D = 0; D < q; ++D)
                    for (int r = 0; r < n; ++r)
                        cbs[((size_t)i * q + D) * n + r] = cb[(size_t)((D + i) % q) * n + r];
            c = mapdec_create_general(q, n, N, cbs.data(), p, p, 0.01, 2, -M, M / 2 + mn,
                                      -mn, mn / 2);
        } else {
            c = mapdec_create(q, n, cb.data(), p, p, 0.01, 2, M, mn);
        }
        if (mode == 2 && f % 4 == 1) {   // path thresholds
            mapdec_code *t = mapdec_with_threshold(c, 1e-9);
            mapdec_destroy(c);
            c = t;
        }
        if (!c) {
            printf("create failed: %s\n", mapdec_strerror(mapdec_last_error()));
            return 1;
        }
        codes.push_back(c);
        int drift = (int)(rng() % (2 * M + 1)) - M;
        if (mode == 2 && f % 3 == 0) drift = drift / 2 > M / 2 + mn ? M / 2 + mn : drift / 2;
        fr[f] = mapdec_frame{c, N, n * N + drift, dev, (!uniform && f % 5 == 0) ? dev : nullptr,
                             dev, dev};
    }
    const size_t ws = mapdec_workspace_size(fr.data(), nf, MAPDEC_FP32, flags, K);
    if (!ws) {
        printf("workspace_size failed\n");
        return 1;
    }
    std::vector<unsigned char> mem(std::min<size_t>(ws, (size_t)256 << 20));
    stub_set_workspace(mem.data(), ws, mem.size(), nf);
    std::vector<double> logp(nf), dparams(3 * nf);
    std::vector<int32_t> status(nf);
    const int live0 = stub_live_objects();
    mapdec_plan *p = mapdec_plan_create(fr.data(), nf, logp.data(), dparams.data(), status.data(),
                                        mem.data(), ws, MAPDEC_FP32, flags, K, nullptr);
    if (!p) {
        printf("plan_create failed: %s\n", mapdec_strerror(mapdec_last_error()));
        return 1;
    }
    for (int r = 0; r < 3; ++r)
        if (mapdec_plan_run(p, nullptr) != MAPDEC_OK) {
            printf("run failed\n");
            return 1;
        }
    float ph[8];
    if (mapdec_plan_profile(p, nullptr, ph, 8) < 0) {
        printf("profile failed\n");
        return 1;
    }
    mapdec_plan_destroy(p);
    if (stub_live_objects() != live0) {
        printf("plan left %d runtime objects behind\n", stub_live_objects() - live0);
        return 1;
    }
    for (mapdec_code *c : codes) mapdec_destroy(c);
    printf("ok frames=%d K=%d flags=%d launches=%ld waits=%ld tuned=%d\n", nf, K, flags,
           stub_launches(), stub_waits(), mapdec_tune_entries());
    return 0;
}

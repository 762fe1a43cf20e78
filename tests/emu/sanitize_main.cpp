// Test-only driver that runs the host planner and the plan emulator on cases
// read from a file, built with AddressSanitizer and UndefinedBehaviorSanitizer
// by tests/test_sanitizers_cpu.py.  Any invalid access or undefined operation
// in the planner (graph analysis, both partition levels, the distributed
// level, lowering) or in the emulated op code aborts the run.
//
// Input (little-endian): int32 n_cases, then per case
//   int32 mode (0 = emulate from |0..0>, 1 = partition only), n, n_gates,
//   n_params, k, R, LW, flags, n_global; qsv_gate[n_gates]; double[n_params].
// Output: per emulated case the complex64 state (2^n pairs of floats); per
// partition-only case int32 n_parts, then per partition uint64 local mask,
// int32 n_gates and the int32 gate indices.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2509_14098_amd/csrc/internal.h"

extern "C" int emu_run_dist(int n, const qsv_gate *gates, int ng, const double *theta, int n_params, int k, int R,
                            int LW, int flags, int inverse, int n_global, float *state);

using namespace qsv;

template <typename T>
static bool get(FILE *f, T *p, size_t count)
{
    return count == 0 || fread(p, sizeof(T), count, f) == count;
}

static int partition_only(FILE *out, int n, const std::vector<qsv_gate> &gates, int n_params, int k, int R, int LW,
                          int flags, int n_global)
{
    Plan P;
    P.n = n;
    P.n_circuits = 1;
    P.k = k < n ? k : n;
    P.t = n < R + LW ? n : R + LW;
    P.R = R;
    P.LW = LW;
    P.flags = (uint32_t)flags;
    if (n_global > 0) {
        P.n_global = n_global;
        distribute(P, gates.data(), (int64_t)gates.size(), n_global);
    } else {
        P.gates = gates;
    }
    CircuitPlan C;
    C.g1 = (int64_t)P.gates.size();
    C.n_params = n_params;
    P.circ.push_back(C);
    P.n_params = n_params;
    build_plan(P);
    const std::vector<Part> &parts = P.circ[0].parts;
    const int32_t np = (int32_t)parts.size();
    fwrite(&np, sizeof(np), 1, out);
    for (const Part &p : parts) {
        const int32_t ng = (int32_t)p.gates.size();
        fwrite(&p.S, sizeof(p.S), 1, out);
        fwrite(&ng, sizeof(ng), 1, out);
        for (int g : p.gates) {
            const int32_t gi = n_global ? (int32_t)P.phys_logical[g] : (int32_t)g;
            fwrite(&gi, sizeof(gi), 1, out);
        }
    }
    return 0;
}

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s cases.bin out.bin\n", argv[0]);
        return 2;
    }
    FILE *in = fopen(argv[1], "rb"), *out = fopen(argv[2], "wb");
    if (!in || !out) return 2;
    int32_t n_cases = 0;
    if (!get(in, &n_cases, 1)) return 3;
    for (int c = 0; c < n_cases; ++c) {
        int32_t h[9];
        if (!get(in, h, 9)) return 3;
        const int mode = h[0], n = h[1], ng = h[2], npar = h[3], k = h[4], R = h[5], LW = h[6], flags = h[7],
                  n_global = h[8];
        std::vector<qsv_gate> gates(ng);
        std::vector<double> theta(npar > 0 ? npar : 1, 0.0);
        if (!get(in, gates.data(), (size_t)ng) || !get(in, theta.data(), (size_t)npar)) return 3;
        if (mode == 0) {
            std::vector<float> state((size_t)2 << n, 0.f);
            state[0] = 1.f;
            emu_run_dist(n, gates.data(), ng, theta.data(), npar, k, R, LW, flags, 0, n_global, state.data());
            fwrite(state.data(), sizeof(float), state.size(), out);
        } else {
            partition_only(out, n, gates, npar, k, R, LW, flags, n_global);
        }
        fprintf(stderr, "case %d done (mode %d, n %d, %d gates)\n", c, mode, n, ng);
    }
    fclose(out);
    fclose(in);
    return 0;
}

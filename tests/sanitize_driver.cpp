// Host-only driver for the sanitizer build of the analysis and the GPU schedule builder
// (kkt_symbolic.cpp, kkt_schedule.cpp compiled with -fsanitize=address,undefined).
// Reads one matrix from a binary file: int32 n, int64 nnz, double tau, int64 rowptr[n+1],
// int32 colind[nnz], double values[nnz]; runs the analysis and the schedule builder and
// prints "status n nnz_lu panels refactor_items solve_items_l solve_items_u".
#include <cstdio>
#include <cstdint>
#include <vector>

#include "../paper_2302_08656_amd/csrc/kkt_internal.h"

int main(int argc, char **argv) {
    if (argc != 2) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t n = 0;
    int64_t nnz = 0;
    double tau = 0.0;
    bool ok = std::fread(&n, 4, 1, f) == 1 && std::fread(&nnz, 8, 1, f) == 1 && std::fread(&tau, 8, 1, f) == 1;
    if (!ok || n < 0 || nnz < 0) return 2;
    std::vector<int64_t> rowptr(n + 1);
    std::vector<int32_t> colind(nnz);
    std::vector<double> vals(nnz);
    ok = std::fread(rowptr.data(), 8, n + 1, f) == (size_t)(n + 1) &&
         std::fread(colind.data(), 4, nnz, f) == (size_t)nnz && std::fread(vals.data(), 8, nnz, f) == (size_t)nnz;
    std::fclose(f);
    if (!ok) return 2;
    kkt_opts o{};
    o.pivot_tau = tau;
    o.tiny_pivot = 1.0 / (1 << 26);
    o.equilibrate = 1;
    o.gmres_restart = 30;
    o.max_iters = 100;
    o.berr_tol = 1e-10;
    o.sn_max_width = 256;
    kkt::Symbolic s;
    kkt::Schedule g;
    int rc = kkt::analyze_symbolic(n, rowptr.data(), colind.data(), vals.data(), o, s);
    if (rc == KKT_OK) rc = kkt::build_schedule(s, kkt::SchedParams{}, g);
    // the other tunable schedules too (narrow panels, fewer narrow rows, small groups)
    for (int32_t pm : {8, 16})
        if (rc == KKT_OK) {
            kkt::Schedule g2;
            rc = kkt::build_schedule(s, kkt::SchedParams{pm, 32, 8}, g2);
        }
    std::printf("%d %d %lld %d %zu %zu %zu\n", rc, n, (long long)s.nnz_lu(), g.npan, g.f_item_panel.size(),
                g.l_item4.size() / 4, g.u_item4.size() / 4);
    return 0;
}

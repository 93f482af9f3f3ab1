// Driver of the CPU emulation: reads one workload written by
// tests/test_emu_kernels.py, runs it through libara's C ABI (compiled for the
// host against the emulated runtime) and writes the year losses, the largest
// occurrence losses and PML/TVaR.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "ara.h"

namespace {
FILE* fin;
template <typename T>
void rd(T* p, size_t n)
{
    if (n && std::fread(p, sizeof(T), n, fin) != n) {
        std::fprintf(stderr, "emu_driver: short input\n");
        std::exit(3);
    }
}
template <typename T>
T rd1()
{
    T v;
    rd(&v, 1);
    return v;
}
void check(ara_ctx* c, ara_status s, const char* what)
{
    if (s != ARA_OK) {
        std::fprintf(stderr, "emu_driver: %s failed (%d): %s\n", what, (int)s, c ? ara_last_error(c) : "");
        std::exit(4);
    }
}
}  // namespace

int main(int argc, char** argv)
{
    if (argc != 3) {
        std::fprintf(stderr, "usage: emu_driver input output\n");
        return 2;
    }
    fin = std::fopen(argv[1], "rb");
    if (!fin) return 2;
    const int64_t N = rd1<int64_t>();
    const int32_t K = rd1<int32_t>(), C = rd1<int32_t>(), has_offs = rd1<int32_t>();
    std::vector<int64_t> offs;
    std::vector<int32_t> ev;
    if (has_offs) {
        offs.resize((size_t)N + 1);
        rd(offs.data(), offs.size());
        ev.resize((size_t)offs.back());
    } else {
        ev.resize((size_t)N * (size_t)K);
    }
    rd(ev.data(), ev.size());
    const int32_t J = rd1<int32_t>();
    std::vector<std::vector<int32_t>> ids(J);
    std::vector<std::vector<double>> mean(J), si(J), sc(J), mx(J);
    std::vector<ara_elt_desc> d(J);
    for (int32_t j = 0; j < J; ++j) {
        const int32_t n = rd1<int32_t>(), has_sc = rd1<int32_t>();
        ids[j].resize(n);
        mean[j].resize(n);
        si[j].resize(n);
        mx[j].resize(n);
        rd(ids[j].data(), n);
        rd(mean[j].data(), n);
        rd(si[j].data(), n);
        if (has_sc) {
            sc[j].resize(n);
            rd(sc[j].data(), n);
        }
        rd(mx[j].data(), n);
        d[j].n_entries = n;
        d[j].event_id = ids[j].data();
        d[j].mean = mean[j].data();
        d[j].sigma_i = si[j].data();
        d[j].sigma_c = has_sc ? sc[j].data() : nullptr;
        d[j].max_loss = mx[j].data();
        d[j].deductible = rd1<double>();
        d[j].limit = rd1<double>();
        d[j].share = rd1<double>();
    }
    ara_layer_desc L{};
    L.n_elts = J;
    L.occ_retention = rd1<double>();
    L.occ_limit = rd1<double>();
    L.agg_retention = rd1<double>();
    L.agg_limit = rd1<double>();
    L.program_id = rd1<uint32_t>();
    const uint32_t seed = rd1<uint32_t>();
    const int32_t mode = rd1<int32_t>(), kind = rd1<int32_t>(), n_rp = rd1<int32_t>();
    std::vector<double> rps(n_rp);
    rd(rps.data(), n_rp);
    std::fclose(fin);

    ara_ctx* c = nullptr;
    check(nullptr, ara_create(0, 0, &c), "ara_create");
    int32_t yh = -1;
    check(c, ara_load_yet(c, ev.data(), has_offs ? offs.data() : nullptr, N, K, C, &yh), "ara_load_yet");
    std::vector<int32_t> eh(J);
    check(c, ara_load_elts(c, C, d.data(), J, eh.data()), "ara_load_elts");
    L.elt_handles = eh.data();
    check(c, ara_set_table_kind(c, kind), "ara_set_table_kind");
    std::vector<float> ylt((size_t)N), omax((size_t)N);
    check(c, ara_run_layer_ex(c, yh, &L, (ara_mode)mode, seed, 0, N, ylt.data(), omax.data(), nullptr),
          "ara_run_layer_ex");
    std::vector<double> pml(n_rp), tvar(n_rp);
    if (n_rp > 0) check(c, ara_risk_measures(c, ylt.data(), N, rps.data(), n_rp, pml.data(), tvar.data(), nullptr),
                        "ara_risk_measures");
    ara_destroy(c);
    FILE* fo = std::fopen(argv[2], "wb");
    if (!fo) return 2;
    std::fwrite(ylt.data(), 4, ylt.size(), fo);
    std::fwrite(omax.data(), 4, omax.size(), fo);
    std::fwrite(pml.data(), 8, pml.size(), fo);
    std::fwrite(tvar.data(), 8, tvar.size(), fo);
    std::fclose(fo);
    return 0;
}

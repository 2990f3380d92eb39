// Host layout under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Reads a problem written by the test as raw little-endian arrays (dir/name.bin),
// lays it out with sim_plan_create for several launch variants and solvers,
// walks every introspection call, and destroys it. Built from the library's
// host source alone: the device launchers, which planning never calls, are
// replaced by stubs below.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../include/sim.h"
#include "../../paper_2005_06332_amd/csrc/internal.h"

namespace mmh {
hipError_t launch_setup(const SetupArgs &, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_epoch(const EpochArgs &, int, int, int, int, size_t, bool, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_fill_u64(uint64_t *, int64_t, uint64_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_advance(int64_t *, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_stamp(uint64_t *, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_decay_weights_convert(const double *, void *, int64_t, int, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t set_epoch_lds_limit(int) { return hipErrorNotSupported; }
hipError_t noalloc_scratch(void **) { return hipErrorNotSupported; }
hipError_t mlp_forward(const float *, const float *, int64_t, float *) { return hipErrorNotSupported; }
hipError_t mlp_loss_grad(const float *, const float *, const float *, int64_t, float *, float *) {
    return hipErrorNotSupported;
}
hipError_t mlp_train(float *, const float *, const float *, int64_t, int, float, float *) {
    return hipErrorNotSupported;
}
}  // namespace mmh

template <typename X>
static std::vector<X> load(const std::string &dir, const char *name) {
    std::string path = dir + "/" + name + ".bin";
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) {
        std::fprintf(stderr, "missing %s\n", path.c_str());
        std::exit(2);
    }
    std::fseek(f, 0, SEEK_END);
    const long bytes = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    std::vector<X> v(bytes / sizeof(X));
    if (!v.empty() && std::fread(v.data(), sizeof(X), v.size(), f) != v.size()) std::exit(2);
    std::fclose(f);
    return v;
}

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    const std::string dir = argv[1];
    auto off = load<int64_t>(dir, "comp_off");
    auto parent = load<int32_t>(dir, "parent");
    auto len = load<double>(dir, "length_um");
    auto diam = load<double>(dir, "diam_um");
    auto mech = load<uint8_t>(dir, "mech");
    auto det = load<int32_t>(dir, "detector");
    auto iext = load<double>(dir, "iext_nA");
    auto pre = load<int32_t>(dir, "syn_pre");
    auto post = load<int32_t>(dir, "syn_post");
    auto comp = load<int32_t>(dir, "syn_comp");
    auto delay = load<int32_t>(dir, "syn_delay");
    auto w = load<double>(dir, "syn_w");
    sim_morphology_t M{(int32_t)off.size() - 1, off.data(), parent.data(), len.data(), diam.data(),
                       mech.data(), det.data(), iext.data()};
    sim_channels_t CH{1.0, 100.0, 0.12, 0.036, 0.0003, 50.0, -77.0, -54.3, 1e-4, -65.0};
    sim_synapses_t SY{(int64_t)pre.size(), pre.data(), post.data(), comp.data(), delay.data(),
                      w.data()};
    int checked = 0;
    for (int solver = 0; solver <= 2; ++solver)
        for (int packing = 0; packing <= 1; ++packing)
            for (int sched : {SIM_SCHED_DISPATCH, SIM_SCHED_PERSISTENT})
                for (int lds_comps : {0, 100}) {
                    sim_params_t P;
                    sim_default_params(&P);
                    P.solver = solver;
                    P.packing = packing;
                    P.sched = sched;
                    P.lds_comps = lds_comps;
                    P.lds_classes = 3;
                    sim_t *s = nullptr;
                    if (sim_plan_create(&P, &M, &CH, &SY, 160 * 1024, 8, &s) != SIM_OK) {
                        std::fprintf(stderr, "plan failed: %s\n", sim_last_error(nullptr));
                        return 1;
                    }
                    const int32_t np = sim_pack_count(s);
                    for (int32_t p = 0; p < np; ++p) {
                        sim_pack_info_t info;
                        if (sim_pack_info(s, p, &info) != SIM_OK) return 1;
                        std::vector<int32_t> ids(info.n_neurons);
                        if (sim_pack_neurons(s, p, ids.data(), (int64_t)ids.size()) != SIM_OK) return 1;
                    }
                    for (int c = 0; c < 3; ++c) {
                        int32_t nwg = 0, thr = 0;
                        int64_t lds = 0;
                        sim_class_launch(s, c, &nwg, &thr, &lds);
                        for (int32_t g = 0; g < nwg; ++g) {
                            int32_t n = 0;
                            sim_workgroup_packs(s, c, g, nullptr, 0, &n);
                            std::vector<int32_t> pk(n > 0 ? n : 1);
                            if (sim_workgroup_packs(s, c, g, pk.data(), n, &n) != SIM_OK) return 1;
                        }
                    }
                    if (solver == 2)
                        for (int32_t pk = 0; pk < sim_pack_count(s); ++pk) {
                            int64_t n = 0;
                            if (sim_pack_contraction_items(s, pk, nullptr, 0, &n) != SIM_OK) return 1;
                            std::vector<uint64_t> items(n > 0 ? n : 1);
                            if (sim_pack_contraction_items(s, pk, items.data(), n, &n) != SIM_OK)
                                return 1;
                        }
                    if (solver == 2)
                        for (int32_t j = 0; j < M.n_neurons; ++j) {
                            int32_t nr = 0;
                            sim_contraction_schedule(s, j, nullptr, 0, nullptr, 0, &nr);
                            const int64_t n = off[j + 1] - off[j];
                            std::vector<int32_t> items(4 * n), ro(nr + 1);
                            if (sim_contraction_schedule(s, j, items.data(), 4 * n, ro.data(), nr + 1,
                                                         &nr) != SIM_OK)
                                return 1;
                        }
                    double v = 0;
                    if (sim_read_voltages(s, &v, 1) != SIM_ESTATE) return 1;
                    sim_destroy(s);
                    ++checked;
                }
    std::printf("planned %d variants\n", checked);
    return 0;
}

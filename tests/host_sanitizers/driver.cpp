// Host-side exercise of the C ABI for a build with AddressSanitizer and UndefinedBehavior-
// Sanitizer on the host code (no GPU is touched: every call below either validates its
// arguments on the host or reports the missing device).  Exit status 0 when every call
// answered as the header documents; the sanitizers abort on any memory or UB error.
#include "lbmix.h"

#include <cstdio>
#include <cstring>
#include <vector>

static int failures = 0;
#define EXPECT(cond)                                                              \
    do {                                                                          \
        if (!(cond)) {                                                            \
            std::fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                           \
        }                                                                         \
    } while (0)

int main(int argc, char **argv) {
    const char *scratch = argc > 1 ? argv[1] : "lbmix_sanitizer_scratch.bin";
    EXPECT(lbmix_version() == 10000);

    lbmix_ctx *c = nullptr;
    EXPECT(lbmix_create(&c, 0, 4, 4, LBMIX_PERIODIC, LBMIX_F32, nullptr) == LBMIX_EINVAL);
    EXPECT(lbmix_create(&c, 4, 4, 2, LBMIX_SLIT_Z, LBMIX_F32, nullptr) == LBMIX_EINVAL);
    EXPECT(lbmix_create(&c, 16384, 8192, 1, LBMIX_PERIODIC, LBMIX_F64, nullptr) == LBMIX_EINVAL);
    EXPECT(lbmix_create(&c, 8, 6, 10, LBMIX_SLIT_Z, LBMIX_F32_SHIFTED, nullptr) == LBMIX_OK);

    int id = -1;
    EXPECT(lbmix_add_species(c, 1.0, 0, &id) == LBMIX_OK && id == 0);
    EXPECT(lbmix_add_species(c, 0.01, 1, &id) == LBMIX_OK && id == 1);
    EXPECT(lbmix_add_species(c, 0.01, -1, &id) == LBMIX_OK && id == 2);
    EXPECT(lbmix_add_species(c, -1.0, 0, &id) == LBMIX_EINVAL);
    EXPECT(lbmix_set_tau_visc(c, 0.5) == LBMIX_EINVAL);
    EXPECT(lbmix_set_tau_visc(c, 0.9) == LBMIX_OK);
    EXPECT(lbmix_set_tau_drag(c, 0.2) == LBMIX_EINVAL);
    EXPECT(lbmix_set_schmidt(c, 10.0) == LBMIX_OK);
    EXPECT(lbmix_set_forcing(c, 7) == LBMIX_EINVAL);
    EXPECT(lbmix_set_forcing(c, LBMIX_FORCING_GUO) == LBMIX_OK);
    EXPECT(lbmix_set_forcing(c, LBMIX_FORCING_PAPER) == LBMIX_OK);
    const double asym[9] = {1.0, 2.0, 3.0, 2.5, 1.0, 2.0, 3.0, 2.0, 1.0};
    EXPECT(lbmix_set_drag_pairs(c, asym) == LBMIX_EINVAL);
    const double sym[9] = {1.0, 2.0, 3.0, 2.0, 1.0, 1.5, 3.0, 1.5, 1.0};
    EXPECT(lbmix_set_drag_pairs(c, sym) == LBMIX_OK);
    EXPECT(lbmix_set_drag_pairs(c, nullptr) == LBMIX_OK);
    const double E[3] = {1e-4, 0.0, 0.0};
    EXPECT(lbmix_set_electrostatics(c, -1.0, 0.0, 0.0, E) == LBMIX_EINVAL);
    EXPECT(lbmix_set_electrostatics(c, 0.6, -1e-4, -1e-4, E) == LBMIX_OK);
    EXPECT(lbmix_set_poisson(c, -1.0, 10, 1, 1.5) == LBMIX_EINVAL);
    EXPECT(lbmix_set_poisson(c, 1e-8, 100, 5, -1.0) == LBMIX_OK);
    EXPECT(lbmix_set_poisson_method(c, 9) == LBMIX_EINVAL);
    EXPECT(lbmix_set_poisson_method(c, 2) == LBMIX_OK);
    EXPECT(lbmix_set_poisson_warm_start(c, 5) == LBMIX_EINVAL);
    EXPECT(lbmix_set_rounding(c, 3, 0) == LBMIX_EINVAL);
    EXPECT(lbmix_set_rounding(c, 1, 42) == LBMIX_OK);
    EXPECT(lbmix_set_storage_range(c, 7, 0.1) == LBMIX_EINVAL);
    EXPECT(lbmix_set_step_graph(c, 1) == LBMIX_OK);

    // no state yet: stepping, reading and saving are refused on the host
    EXPECT(lbmix_step(c, 1) == LBMIX_ESTATE);
    EXPECT(lbmix_autotune(c, 2) == LBMIX_ESTATE);
    std::vector<double> buf(8 * 6 * 10 * 19, 0.0);
    EXPECT(lbmix_get_moments(c, 0, buf.data(), nullptr) == LBMIX_ESTATE);
    EXPECT(lbmix_get_mass_totals(c, buf.data()) == LBMIX_ESTATE);
    EXPECT(lbmix_get_step_mass(c, buf.data()) == LBMIX_ESTATE);
    EXPECT(lbmix_get_step_mass(nullptr, buf.data()) == LBMIX_EINVAL);
    EXPECT(lbmix_save(c, scratch) == LBMIX_ESTATE);
    EXPECT(std::strlen(lbmix_last_error(c)) > 0);
    lbmix_stats st;
    EXPECT(lbmix_get_stats(c, &st) == LBMIX_OK);
    EXPECT(st.steps == 0);

    // a file that is not a checkpoint, and one that does not exist
    if (FILE *fp = std::fopen(scratch, "wb")) {
        const char junk[64] = "not a checkpoint";
        std::fwrite(junk, 1, sizeof junk, fp);
        std::fclose(fp);
    }
    EXPECT(lbmix_load(c, scratch) == LBMIX_EINVAL);
    std::remove(scratch);
    EXPECT(lbmix_load(c, scratch) == LBMIX_EINVAL);

    // the first device call reports the missing GPU (on a GPU host it allocates instead)
    std::vector<double> n(8 * 6 * 10, 1.0);
    const int rc = lbmix_set_state(c, 0, n.data(), nullptr);
    EXPECT(rc == LBMIX_EDEVICE || rc == LBMIX_OK);
    lbmix_destroy(c);
    lbmix_destroy(nullptr);

    // channel stacks
    const int widths[3] = {4, 5, 6};
    EXPECT(lbmix_create_channels(&c, 8, 8, 0, widths, LBMIX_F32_SHIFTED, nullptr) == LBMIX_EINVAL);
    EXPECT(lbmix_create_channels(&c, 8, 8, 3, widths, LBMIX_F32_SHIFTED, nullptr) == LBMIX_OK);
    EXPECT(lbmix_set_channel(c, 3, 0.7, 0.0, 0.0) == LBMIX_EINVAL);
    EXPECT(lbmix_set_channel(c, 1, 0.7, -1e-4, -2e-4) == LBMIX_OK);
    lbmix_destroy(c);

    // warm-start networks: host-side validation only
    lbmix_net *net = nullptr;
    EXPECT(lbmix_net_create(&net, 0, 16, 3, 1) == LBMIX_EINVAL);
    EXPECT(lbmix_net_create(&net, 4, 64, 3, 1) == LBMIX_EINVAL);
    const int nr = lbmix_net_create(&net, 4, 16, 3, 1);
    EXPECT(nr == LBMIX_OK || nr == LBMIX_EDEVICE);
    if (nr == LBMIX_OK) {
        EXPECT(lbmix_net_num_params(net) > 0);
        EXPECT(lbmix_net_forward(net, nullptr, nullptr, 4, 4, 4, 0, nullptr) == LBMIX_EINVAL);
        EXPECT(lbmix_net_forward_noalloc(net, nullptr, nullptr, 4, 4, 4, 0, nullptr) == LBMIX_EINVAL);
        lbmix_net_destroy(net);
    }
    lbmix_net_destroy(nullptr);
    EXPECT(lbmix_net_forward_noalloc(nullptr, nullptr, nullptr, 4, 4, 4, 0, nullptr) == LBMIX_EINVAL);

    if (failures) std::fprintf(stderr, "%d expectation(s) failed\n", failures);
    else std::printf("host ABI checks passed\n");
    return failures ? 1 : 0;
}

// Host-side check of the C ABI under AddressSanitizer and UBSan: every entry
// point with null or invalid arguments, the state errors, the option checks
// and, when no device is present, the HIP error path of context and server
// creation.  Built host-only by tests/test_sanitizers.py (no kernel runs).
#include <cstdio>
#include <cstring>

#include "mdwf.h"

static int failures = 0;
#define EXPECT(cond)                                               \
    do {                                                           \
        if (!(cond)) {                                             \
            std::printf("FAILED: %s (line %d)\n", #cond, __LINE__); \
            ++failures;                                            \
        }                                                          \
    } while (0)

int main() {
    mdwf_ctx* c = nullptr;
    EXPECT(mdwf_create(nullptr, 0, nullptr, &c) == MDWF_ERR_ARG);
    mdwf_geometry odd{4, 3, 4, 4, 1}, zero{4, 4, 0, 4, 1}, good{4, 4, 4, 8, 1};
    EXPECT(mdwf_create(&odd, 0, nullptr, &c) == MDWF_ERR_ARG);
    EXPECT(mdwf_create(&zero, 0, nullptr, &c) == MDWF_ERR_ARG);
    EXPECT(mdwf_create(&good, 0, nullptr, nullptr) == MDWF_ERR_ARG);
    EXPECT(std::strlen(mdwf_last_error(nullptr)) > 0);
    mdwf_destroy(nullptr);

    mdwf_action act{1.3, 1.5, 0.5, 0.05, 8};
    mdwf_solver_opts o;
    mdwf_default_opts(&o);
    mdwf_default_opts(nullptr);
    EXPECT(o.tol == 1e-10 && o.inner == MDWF_F64 && o.schur_form == 0 && o.max_seconds == 0.0);
    double d = 0.0, f = 0.0;
    size_t nb = 0;
    mdwf_launch_tune tune[3];
    mdwf_solve_info info[2];
    const double* bs[1] = {&d};
    double* xs[1] = {&d};
    EXPECT(mdwf_set_action(nullptr, &act) == MDWF_ERR_ARG);
    EXPECT(mdwf_load_gauge(nullptr, &d) == MDWF_ERR_ARG);
    EXPECT(mdwf_load_gauge_dev(nullptr, &d) == MDWF_ERR_ARG);
    EXPECT(mdwf_field_bytes(nullptr, MDWF_F32, MDWF_FULL, &nb) == MDWF_ERR_ARG);
    EXPECT(mdwf_pack_dev(nullptr, MDWF_F32, MDWF_FULL, &d, &f, nullptr) == MDWF_ERR_ARG);
    EXPECT(mdwf_unpack_dev(nullptr, MDWF_F32, MDWF_FULL, &f, &d, nullptr) == MDWF_ERR_ARG);
    EXPECT(mdwf_apply(nullptr, MDWF_OP_SCHUR, MDWF_F64, &d, &f) == MDWF_ERR_ARG);
    EXPECT(mdwf_apply_dev(nullptr, MDWF_OP_SCHUR_RP, MDWF_F16, &d, &f, nullptr) == MDWF_ERR_ARG);
    EXPECT(mdwf_solve(nullptr, 1, bs, xs, nullptr, &o, info) == MDWF_ERR_ARG);
    EXPECT(mdwf_solve_dev(nullptr, 1, bs, xs, nullptr, &o, info, nullptr) == MDWF_ERR_ARG);
    EXPECT(mdwf_autotune(nullptr, tune) == MDWF_ERR_ARG);
    EXPECT(mdwf_autotune_solve(nullptr, &o, 2, tune) == MDWF_ERR_ARG);
    EXPECT(mdwf_get_tune(nullptr, MDWF_F16, tune) == MDWF_ERR_ARG);
    EXPECT(mdwf_op_model(nullptr, MDWF_OP_SCHUR, MDWF_F32, &d, &f) == MDWF_ERR_ARG);

    // sources, sinks and flow: argument errors are found before any HIP call
    double buf[16] = {0}, cpp[8], cmp[8], mres[8], plaq[2];
    mdwf_geometry flat{4, 4, 0, 8, 1}, tall{1, 1, 1, 70000, 1};
    EXPECT(mdwf_gauss_smear_dev(nullptr, buf, 1, buf, buf + 8, 2.0, 3, nullptr) == MDWF_ERR_ARG);
    EXPECT(mdwf_gauss_smear_dev(&flat, buf, 1, buf, buf + 8, 2.0, 3, nullptr) == MDWF_ERR_ARG);
    EXPECT(mdwf_gauss_smear_dev(&good, buf, 1, buf, buf + 1, 2.0, 3, nullptr) == MDWF_ERR_ARG);   // overlap
    EXPECT(mdwf_gauss_smear_dev(&good, buf, 0, buf, buf + 8, 2.0, 3, nullptr) == MDWF_ERR_ARG);
    EXPECT(mdwf_wall_source_dev(&good, nullptr, buf, 1, buf, buf + 8, nullptr) == MDWF_ERR_ARG);
    mdwf_action l0 = act;
    l0.L5 = 0;
    EXPECT(mdwf_wall_source_dev(&good, &l0, buf, 1, buf, buf + 8, nullptr) == MDWF_ERR_ARG);
    EXPECT(mdwf_project_4d_dev(&good, 5, 1, buf, buf + 8, buf + 4, nullptr) == MDWF_ERR_ARG);
    EXPECT(mdwf_mres_correlators_dev(&good, 7, 1, buf, nullptr, cpp, cmp, mres) == MDWF_ERR_ARG);
    EXPECT(mdwf_mres_correlators_dev(&tall, 8, 1, buf, nullptr, cpp, cmp, mres) == MDWF_ERR_ARG);
    EXPECT(mdwf_pion_correlator_dev(&tall, 1, buf, nullptr, cpp) == MDWF_ERR_ARG);
    EXPECT(mdwf_pion_correlator_dev(&good, 0, buf, nullptr, cpp) == MDWF_ERR_ARG);
    EXPECT(mdwf_wilson_flow_dev(&good, buf, -1.0, 2, nullptr, plaq) == MDWF_ERR_ARG);
    EXPECT(mdwf_wilson_flow(&flat, 0, buf, 0.01, 2, plaq) == MDWF_ERR_ARG);
    EXPECT(mdwf_plaquette_dev(&good, nullptr, nullptr, plaq) == MDWF_ERR_ARG);

    // a context: on a host with a device the state and argument errors
    // follow; without one, creation reports the HIP error
    const mdwf_status cs = mdwf_create(&good, 0, nullptr, &c);
    EXPECT(cs == MDWF_OK || cs == MDWF_ERR_HIP);
    if (cs == MDWF_OK) {
        EXPECT(mdwf_solve(c, 1, bs, xs, nullptr, &o, info) == MDWF_ERR_STATE);
        mdwf_action bad = act;
        bad.L5 = 0;
        EXPECT(mdwf_set_action(c, &bad) == MDWF_ERR_ARG);
        bad = act;
        bad.c5 = bad.b5;
        EXPECT(mdwf_set_action(c, &bad) == MDWF_ERR_ARG);
        bad = act;
        bad.mq = -0.1;
        EXPECT(mdwf_set_action(c, &bad) == MDWF_ERR_ARG);
        EXPECT(mdwf_set_action(c, &act) == MDWF_OK);
        EXPECT(mdwf_apply(c, MDWF_OP_D5, MDWF_F64, &d, &f) == MDWF_ERR_STATE);
        mdwf_destroy(c);
    }

    // server
    mdwf_server* s = nullptr;
    int id = 0;
    size_t b1 = 0, b2 = 0;
    int q = 0;
    EXPECT(mdwf_server_create(0, 0, 0, &s) == MDWF_ERR_ARG);
    EXPECT(mdwf_server_create(0, 0, 2, nullptr) == MDWF_ERR_ARG);
    EXPECT(mdwf_server_add_field(nullptr, &good, &d, &id) == MDWF_ERR_ARG);
    EXPECT(mdwf_server_submit(nullptr, 0, &act, 1, bs, xs, nullptr, &o, &id) == MDWF_ERR_ARG);
    EXPECT(mdwf_server_wait(nullptr, 1, info, nullptr) == MDWF_ERR_ARG);
    EXPECT(mdwf_server_stats(nullptr, &b1, &b2, &q) == MDWF_ERR_ARG);
    EXPECT(mdwf_server_last_error(nullptr) != nullptr);
    mdwf_server_destroy(nullptr);
    const mdwf_status ss = mdwf_server_create(0, 1 << 30, 2, &s);
    EXPECT(ss == MDWF_OK || ss == MDWF_ERR_HIP);
    if (ss == MDWF_OK) {
        EXPECT(mdwf_server_submit(s, 3, &act, 1, bs, xs, nullptr, &o, &id) == MDWF_ERR_ARG);   // no such field
        EXPECT(mdwf_server_wait(s, 99, info, nullptr) == MDWF_ERR_ARG);
        EXPECT(mdwf_server_stats(s, &b1, &b2, &q) == MDWF_OK && q == 0);
        mdwf_server_destroy(s);
    }
    std::printf(failures ? "abi sanitizer run: FAILED\n" : "abi sanitizer run: ok\n");
    return failures ? 1 : 0;
}

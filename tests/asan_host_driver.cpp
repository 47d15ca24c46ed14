// Host-side paths of liblbm under AddressSanitizer and UndefinedBehaviorSanitizer
// (TEST INFRASTRUCTURE: built host-only by tests/test_host_sanitizers.py, no device
// code and no device needed): the plan and workspace sizing over a grid of valid
// and invalid parameters, the argument checks of every entry point that can fail
// before touching a device, the multipole expansion with its closed-form checks,
// the status strings and the checkpoint sizing guard.  Exits non-zero on the first
// failed check; the sanitizers abort on the first memory or UB error.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <random>
#include <vector>

#include "../include/lbm.h"

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);   \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

static void sizing()
{
    const int dims[] = {2, 4, 5, 7, 16, 33, 64, 130};
    const int tiles[][3] = {{0, 0, 0}, {64, 2, 2}, {16, 4, 4}, {256, 1, 1}, {64, 3, 1}, {128, 1, 2}, {8, 8, 8}};
    const int variants[] = {0, 2, 16, 32, 54, 66, 194, 255, 256, -1};
    const long long points[] = {0, 1, 1000, (1LL << 23), (1LL << 24), -3};
    std::vector<double> tau(5, 0.8);
    long ok = 0, bad = 0;
    for (int nx : dims)
        for (int ny : {4, 9})
            for (int nz : {4, 6})
                for (int st = -1; st <= 4; ++st)
                    for (auto& t : tiles)
                        for (int v : variants)
                            for (long long mp : points)
                                for (int coll = 0; coll <= 3; ++coll) {
                                    lb_params p;
                                    memset(&p, 0, sizeof(p));
                                    p.nx = nx; p.ny = ny; p.nz = nz;
                                    p.nboxes = (nx % 3) + 1;
                                    p.storage = st;
                                    p.tau = tau.data();
                                    p.max_points = mp;
                                    p.tile_x = t[0]; p.tile_y = t[1]; p.tile_z = t[2];
                                    p.variant = v;
                                    p.collision = coll;
                                    p.ghost_rate = coll == 2 ? 1.5 : 2.0;
                                    size_t b = 0;
                                    const int r = lb_workspace_bytes(&p, &b);
                                    CHECK(r == LB_OK || r == LB_ERR_ARG || r == LB_ERR_SIZE);
                                    if (r == LB_OK) {
                                        ++ok;
                                        const size_t pops = 2ull * nx * ny * nz * p.nboxes;
                                        CHECK(b >= pops * (st == LB_STORAGE_FP16 ? 2 : 4));
                                    } else {
                                        ++bad;
                                        CHECK(strlen(lb_last_error(nullptr)) > 0);
                                    }
                                }
    size_t b = 0;
    CHECK(lb_workspace_bytes(nullptr, &b) == LB_ERR_ARG);
    printf("sizing: %ld accepted, %ld rejected parameter sets\n", ok, bad);
    CHECK(ok > 0 && bad > 0);
}

static void entry_argument_checks()
{
    lb_params p;
    memset(&p, 0, sizeof(p));
    p.nx = p.ny = p.nz = 8;
    p.nboxes = 1;
    double tau = 0.7;
    p.tau = &tau;
    CHECK(lb_init(&p, nullptr, 0, nullptr, nullptr) == LB_ERR_ARG);
    CHECK(lb_set_stream(nullptr, nullptr) == LB_ERR_ARG);
    CHECK(lb_step(nullptr, 1) == LB_ERR_ARG);
    CHECK(lb_prepare_steps(nullptr, 8) == LB_ERR_ARG);
    CHECK(lb_moments(nullptr, nullptr, nullptr) == LB_ERR_ARG);
    CHECK(lb_interp_velocity(nullptr, 1, nullptr, nullptr, nullptr) == LB_ERR_ARG);
    CHECK(lb_add_point_forces(nullptr, 1, nullptr, nullptr, nullptr, LB_FORCES_STATIC, nullptr) == LB_ERR_ARG);
    CHECK(lb_add_elastic(nullptr, nullptr) == LB_ERR_ARG);
    CHECK(lb_clear_forces(nullptr) == LB_ERR_ARG);
    CHECK(lb_diagnostics(nullptr, nullptr) == LB_ERR_ARG);
    CHECK(lb_sync(nullptr) == LB_ERR_ARG);
    CHECK(lb_destroy(nullptr) == LB_ERR_ARG);
    CHECK(lb_kernel_timing(nullptr, 1) == LB_ERR_ARG);
    CHECK(lb_kernel_time(nullptr, nullptr, nullptr) == LB_ERR_ARG);
    CHECK(lb_steps_taken(nullptr) == -1);
    size_t b = 0;
    CHECK(lb_checkpoint_bytes(nullptr, &b) == LB_ERR_ARG);
    CHECK(lb_checkpoint_save(nullptr, nullptr) == LB_ERR_ARG);
    CHECK(lb_checkpoint_load(nullptr, nullptr) == LB_ERR_ARG);
    CHECK(lb_copy_probe(nullptr, nullptr, 16, nullptr) == LB_ERR_ARG);
    CHECK(lbml_work_floats(-1) == -1 && lbml_work_floats(10) == 2580);
    CHECK(lbml_round_bf16(nullptr, nullptr, nullptr) == LB_ERR_ARG);
    CHECK(lbml_forward(nullptr, 4, nullptr, nullptr, nullptr) == LB_ERR_ARG);
    CHECK(lbml_forward(nullptr, 0, nullptr, nullptr, nullptr) == LB_OK);
    CHECK(lbml_loss_grad(nullptr, 4, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == LB_ERR_ARG);
    CHECK(lbml_loss_grad_static(nullptr, 4, nullptr, nullptr, nullptr, nullptr, nullptr) == LB_ERR_ARG);
    CHECK(lbml_adam_step(nullptr, nullptr, nullptr, nullptr, nullptr, 1, 1e-3f, 0.9f, 0.999f, 1e-8f, nullptr) ==
          LB_ERR_ARG);
    for (int s = -9; s <= 1; ++s) CHECK(strlen(lb_status_string(s)) > 0);
    CHECK(strcmp(lb_status_string(12345), "unknown status") == 0);
}

static void multipoles()
{
    std::mt19937_64 g(7);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    for (int n : {0, 1, 5, 64}) {
        std::vector<int32_t> type(n);
        std::vector<double> c(3 * n), ax(3 * n), e1(3 * n), s(n);
        for (int i = 0; i < n; ++i) {
            type[i] = i % 3;
            double a[3] = {u(g), u(g), u(g) + 2.0}, e[3] = {u(g), u(g), u(g)};
            const double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
            for (int k = 0; k < 3; ++k) a[k] /= la;
            const double d = e[0] * a[0] + e[1] * a[1] + e[2] * a[2];
            for (int k = 0; k < 3; ++k) e[k] -= d * a[k];
            const double le = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
            for (int k = 0; k < 3; ++k) {
                ax[3 * i + k] = a[k];
                e1[3 * i + k] = e[k] / le;
                c[3 * i + k] = 10.0 * u(g);
            }
            s[i] = u(g) * 1e-5;
        }
        std::vector<double> pos(12 * (size_t)n + 3), frc(12 * (size_t)n + 3);
        int64_t m = -1;
        CHECK(lb_expand_multipoles(n, type.data(), c.data(), ax.data(), e1.data(), s.data(), 2.0, &m, pos.data(),
                                   frc.data()) == LB_OK);
        int64_t want = 0;
        for (int i = 0; i < n; ++i) want += type[i] == 0 ? 1 : (type[i] == 1 ? 2 : 4);
        CHECK(m == want);
        // net force of each multipole: s p for a Stokeslet, zero for the others
        int64_t o = 0;
        for (int i = 0; i < n; ++i) {
            const int k = type[i] == 0 ? 1 : (type[i] == 1 ? 2 : 4);
            for (int a = 0; a < 3; ++a) {
                double f = 0.0;
                for (int j = 0; j < k; ++j) f += frc[3 * (o + j) + a];
                CHECK(fabs(f - (type[i] == 0 ? s[i] * ax[3 * i + a] : 0.0)) < 1e-20);
            }
            o += k;
        }
    }
    int32_t bad_type = 7;
    double z[3] = {0, 0, 1}, pos[12], frc[12];
    int64_t m = 0;
    CHECK(lb_expand_multipoles(1, &bad_type, z, z, z, z, 2.0, &m, pos, frc) == LB_ERR_ARG);
    CHECK(lb_expand_multipoles(-1, nullptr, nullptr, nullptr, nullptr, nullptr, 2.0, &m, nullptr, nullptr) ==
          LB_ERR_ARG);
}

int main()
{
    sizing();
    entry_argument_checks();
    multipoles();
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("host checks passed\n");
    return 0;
}

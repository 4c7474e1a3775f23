// Host-side paths of the C ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer (host code only; the device is never touched):
// parameter validation of every field, workspace layouts of every model,
// context creation and destruction, call-order checks, the stateless and
// static-scratch entry points' argument checks, batch creation checks and
// the thread-local error strings.  Exit status 0 when every call returned
// the expected status.
#include <stdio.h>
#include <string.h>

#include "../../include/sobrc.h"

static int failures = 0;
#define EXPECT(cond)                                                       \
    do {                                                                   \
        if (!(cond)) {                                                     \
            fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static sobrc_params base2d()
{
    sobrc_params p;
    memset(&p, 0, sizeof p);
    p.ndim = 2; p.nx = 64; p.ny = 48; p.nz = 1;
    p.image_dtype = SOBRC_F32; p.model = SOBRC_PC; p.ps_radius = 0;
    p.E = 8.0; p.eps = 1.0 / 24.0; p.lambda = 0.1;
    p.max_labels = 2; p.max_particles = 1000;
    p.noise = SOBRC_NOISE_GAUSS; p.topo = SOBRC_TOPO_OFF; p.psf_sigma = 0.0;
    return p;
}

int main()
{
    size_t n = 0;
    // every rejected field
    for (int k = 0; k < 16; ++k) {
        sobrc_params p = base2d();
        switch (k) {
        case 0: p.ndim = 4; break;
        case 1: p.nx = 0; break;
        case 2: p.ny = 40000; break;
        case 3: p.nz = 2; break;
        case 4: p.image_dtype = 7; break;
        case 5: p.model = 3; break;
        case 6: p.model = SOBRC_PS; p.ps_radius = 1; break;
        case 7: p.E = 0.0; break;
        case 8: p.eps = 0.0; break;
        case 9: p.lambda = -1.0; break;
        case 10: p.max_labels = 1; break;
        case 11: p.max_particles = 0; break;
        case 12: p.noise = 2; break;
        case 13: p.topo = 2; break;
        case 14: p.psf_sigma = 16.5; break;
        case 15: p.psf_sigma = 2.0; p.max_labels = 5; break;
        }
        EXPECT(workspace_size(&p, &n) == SOBRC_EINVAL);
        EXPECT(last_error() != nullptr && strlen(last_error()) > 0);
    }
    EXPECT(workspace_size(nullptr, &n) == SOBRC_EINVAL);
    // layouts of every model and dimension
    const int dims[][4] = {{2, 64, 48, 1}, {3, 40, 33, 27}, {2, 1, 1, 1}, {3, 1, 1, 1}, {3, 1024, 8, 8}};
    for (auto& d : dims)
        for (int variant = 0; variant < 5; ++variant) {
            sobrc_params p = base2d();
            p.ndim = d[0]; p.nx = d[1]; p.ny = d[2]; p.nz = d[3];
            p.image_dtype = variant == 1 ? SOBRC_U16 : SOBRC_F32;
            if (variant == 2) { p.model = SOBRC_PS; p.ps_radius = 4; }
            if (variant == 3) p.topo = SOBRC_TOPO_SIMPLE;
            if (variant == 4) { p.psf_sigma = 1.5; p.max_labels = 3; }
            EXPECT(workspace_size(&p, &n) == SOBRC_OK && n > 0);
            size_t ns = 0;
            EXPECT(sobolev_particles_workspace_size(&p, 100, &ns) == SOBRC_OK && ns > 0);
            // a context in a fake workspace: created and destroyed without device calls
            sobrc_ctx* h = nullptr;
            void* fake = (void*)(uintptr_t)(1u << 20);
            EXPECT(ctx_create(&p, nullptr, n, &h) == SOBRC_EINVAL);
            EXPECT(ctx_create(&p, (void*)((uintptr_t)(1u << 20) + 4), n, &h) == SOBRC_EINVAL);
            EXPECT(ctx_create(&p, fake, n - 1, &h) == SOBRC_EINVAL);
            EXPECT(ctx_create(&p, fake, n, &h) == SOBRC_OK && h != nullptr);
            float* ff = (float*)fake;
            EXPECT(step(h, SOBRC_MODE_SOBOLEV, nullptr, nullptr) == SOBRC_ESTATE);
            EXPECT(run(h, 3, 0.0, SOBRC_MODE_SOBOLEV, nullptr, nullptr) == SOBRC_ESTATE);
            EXPECT(compute_l2_diff(h, ff, nullptr) == SOBRC_ESTATE);
            EXPECT(sobolev_smooth(h, ff, ff + 1, nullptr) == SOBRC_ESTATE);
            EXPECT(step_with_gradient(h, ff, nullptr, nullptr) == SOBRC_ESTATE);
            EXPECT(init_labels(h, nullptr, (const int32_t*)fake, nullptr) == SOBRC_EINVAL);
            EXPECT(ctx_destroy(h) == SOBRC_OK);
        }
    EXPECT(ctx_destroy(nullptr) == SOBRC_EINVAL);
    // stateless entry points: argument checks before any device call
    {
        sobrc_params p = base2d();
        void* fake = (void*)(uintptr_t)(1u << 20);
        const int32_t* fi = (const int32_t*)fake;
        EXPECT(sobolev_smooth_particles(&p, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) ==
               SOBRC_OK);
        EXPECT(sobolev_smooth_particles(&p, 10, fi, fi, fi, (const float*)fake, (float*)fake, fake, 16, nullptr) ==
               SOBRC_EINVAL);
        EXPECT(sobolev_smooth_particles_static(&p, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
               SOBRC_OK);
        EXPECT(sobolev_smooth_particles_static(&p, 4 << 20, fi, fi, fi, (const float*)fake, (float*)fake,
                                               nullptr) == SOBRC_EINVAL);
        EXPECT(sobolev_smooth_particles_static(&p, -1, fi, fi, fi, (const float*)fake, (float*)fake, nullptr) ==
               SOBRC_EINVAL);
    }
    // batches
    {
        size_t nb = 0;
        EXPECT(batch_workspace_size(0, &nb) == SOBRC_EINVAL);
        EXPECT(batch_workspace_size(4, &nb) == SOBRC_OK);
        sobrc_batch* B = nullptr;
        EXPECT(batch_create(4, nullptr, nb, &B) == SOBRC_EINVAL);
        EXPECT(batch_create(4, (void*)0x1001, nb, &B) == SOBRC_EINVAL);
        EXPECT(batch_create(4, (void*)0x10000, 16, &B) == SOBRC_EINVAL);
        EXPECT(batch_destroy(nullptr) == SOBRC_EINVAL);
        EXPECT(batch_set(nullptr, 0, nullptr, nullptr) == SOBRC_EINVAL);
        EXPECT(batch_run(nullptr, 1, 0.0, 0, nullptr, nullptr) == SOBRC_EINVAL);
    }
    if (failures)
        return 1;
    printf("abi driver: all host-side checks passed\n");
    return 0;
}

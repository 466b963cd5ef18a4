/*
 * Drives the validation layer of the C ABI (include/fsr.h) without a GPU:
 * every call below is refused before anything touches a device, so a build
 * of the library's host code with AddressSanitizer and
 * UndefinedBehaviorSanitizer can check it on any machine (test
 * infrastructure; built by tests/test_sanitizers.py).
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "fsr.h"

#define EXPECT(cond)                                                     \
    do {                                                                 \
        if (!(cond)) {                                                   \
            printf("FAILED: %s (line %d)\n", #cond, __LINE__);           \
            return 1;                                                    \
        }                                                                \
    } while (0)

int main(void)
{
    fsr_params p;
    EXPECT(fsr_params_default(&p) == FSR_OK);
    EXPECT(fsr_params_validate(&p) == FSR_OK);
    EXPECT(fsr_params_default(NULL) == FSR_ERR_INVALID_ARG);
    fsr_params bad = p;
    bad.rho = 0.0f;
    EXPECT(fsr_params_validate(&bad) == FSR_ERR_INVALID_ARG);
    EXPECT(strlen(fsr_last_error_message()) > 0);
    EXPECT(fsr_num_blocks(1080, 1920, 4) == 129600);
    EXPECT(fsr_num_blocks(0, 1, 4) == -1);
    for (int s = -1; s <= 8; ++s) EXPECT(fsr_status_string(s) != NULL);
    EXPECT(strcmp(fsr_status_string(99), "FSR_ERR_UNKNOWN") == 0);

    fsr_context *ctx = (fsr_context *)(uintptr_t)0x1000;   /* never dereferenced */
    const float *img = (const float *)(uintptr_t)0x10000;
    const uint8_t *msk = (const uint8_t *)(uintptr_t)0x20000000;
    float *out = (float *)(uintptr_t)0x40000000;
    EXPECT(fsr_reconstruct(NULL, img, msk, out, 8, 8, 8, &p, NULL, NULL) == FSR_ERR_INVALID_ARG);
    EXPECT(fsr_reconstruct(ctx, img, msk, out, 8, 8, 7, &p, NULL, NULL) == FSR_ERR_INVALID_ARG);
    EXPECT(fsr_reconstruct(ctx, img, msk, (float *)(uintptr_t)0x10040, 8, 8, 8, &p, NULL, NULL) ==
           FSR_ERR_INVALID_ARG);
    fsr_params p12 = p;
    p12.border = 4;
    EXPECT(fsr_reconstruct(ctx, img, msk, out, 8, 8, 8, &p12, NULL, NULL) == FSR_ERR_UNSUPPORTED);
    EXPECT(fsr_reconstruct_reuse(ctx, img, msk, out, 8, 8, 8, &p, 1.5f, NULL, NULL) == FSR_ERR_INVALID_ARG);
    EXPECT(fsr_reconstruct_reuse_frames(ctx, img, msk, out, 0, 8, 8, 8, 64, &p, 0.5f, NULL, NULL) ==
           FSR_ERR_INVALID_ARG);
    EXPECT(fsr_reconstruct_reuse_frames(ctx, img, msk, out, 2, 8, 8, 8, 63, &p, 0.5f, NULL, NULL) ==
           FSR_ERR_INVALID_ARG);

    size_t bytes = 0;
    EXPECT(fsr_batched_workspace_size(4, &bytes) == FSR_OK && bytes > 0);
    EXPECT(fsr_batched_workspace_size(-1, &bytes) == FSR_ERR_INVALID_ARG);
    fsr_image_desc d;
    memset(&d, 0, sizeof d);
    EXPECT(fsr_reconstruct_batched(ctx, &d, 1, &p, NULL, NULL, 0, NULL) == FSR_ERR_INVALID_ARG);

    fsr_server_config cfg;
    memset(&cfg, 0, sizeof cfg);
    fsr_server *srv = NULL;
    EXPECT(fsr_server_create(ctx, &p, &cfg, &srv) == FSR_ERR_INVALID_ARG && srv == NULL);
    printf("abi validation clean\n");
    return 0;
}

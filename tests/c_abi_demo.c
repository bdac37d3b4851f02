/* Plain-C use of the library through include/kerrtrace.h and the HIP runtime
 * API alone (no Python, no torch): renders the 64x64 Schwarzschild shadow
 * (a = 0, r_obs = 1000M, i = 90 deg, +-10M, fixed-step RK4 in s with
 * h_s = 1/128, capture below 2.01M, escape beyond 1100M) and prints the
 * number of captured pixels.  Synge's shadow x^2 + y^2 < 27 M^2 (1 - 2M/r_obs)
 * holds 872 pixel centres of this grid.
 *
 *   c_abi_demo --version   prints kt_version() (no GPU needed)
 *   c_abi_demo             renders on device 0; exit status 0 iff 872 captured
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "kerrtrace.h"

#define CHECK_HIP(x)                                                           \
    do {                                                                       \
        hipError_t e_ = (x);                                                   \
        if (e_ != hipSuccess) {                                                \
            fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));     \
            return 2;                                                          \
        }                                                                      \
    } while (0)

int main(int argc, char **argv) {
    if (argc > 1 && strcmp(argv[1], "--version") == 0) {
        printf("%d\n", kt_version());
        return kt_version() == KT_VERSION_NUMBER ? 0 : 1;
    }
    kt_camera cam = {1000.0, 1.5707963267948966, 10.0, 10.0, 64, 64};
    kt_spacetime st = {1.0, 0.0, KT_METRIC_KERR, 0.0};
    kt_integrator integ;
    memset(&integ, 0, sizeof integ);
    integ.method = KT_RK4_S;
    integ.precision = KT_FP64;
    integ.h_fixed = 1.0 / 128;
    integ.capture_buffer = 0.01;
    integ.r_escape = 1100.0;
    integ.max_steps = 1000000;
    const size_t n = (size_t)cam.nx * (size_t)cam.ny;

    kt_outputs out;
    memset(&out, 0, sizeof out);
    void *fate = NULL, *ws = NULL;
    CHECK_HIP(hipMalloc(&fate, n));
    out.fate = (uint8_t *)fate;
    const size_t ws_bytes = kt_workspace_bytes(&cam, &integ);
    if (ws_bytes == 0) {
        fprintf(stderr, "kt_workspace_bytes: %s\n", kt_last_error());
        return 2;
    }
    CHECK_HIP(hipMalloc(&ws, ws_bytes)); /* hipMalloc returns 256-byte-aligned memory */

    const int rc = kt_render(&cam, &st, NULL, NULL, &integ, &out, ws, ws_bytes, NULL);
    if (rc != KT_OK) {
        fprintf(stderr, "kt_render: %d %s\n", rc, kt_last_error());
        return 2;
    }
    CHECK_HIP(hipDeviceSynchronize());
    uint8_t *host = (uint8_t *)malloc(n);
    CHECK_HIP(hipMemcpy(host, fate, n, hipMemcpyDeviceToHost));
    size_t captured = 0, escaped = 0;
    for (size_t k = 0; k < n; ++k) {
        captured += host[k] == KT_FATE_CAPTURED;
        escaped += host[k] == KT_FATE_ESCAPED;
    }
    printf("captured %zu escaped %zu of %zu\n", captured, escaped, n);
    free(host);
    CHECK_HIP(hipFree(fate));
    CHECK_HIP(hipFree(ws));
    return captured == 872 && captured + escaped == n ? 0 : 1;
}

// Exercises the host-only calls of the C ABI (cosmology factors, halt predicate, forecast)
// on valid and invalid arguments, for an AddressSanitizer + UndefinedBehaviorSanitizer build
// of the library's host source (test infrastructure, CPU only).  Exits 0 when every call
// returned the expected status; the sanitizers abort on the first finding.
#include <math.h>
#include <stdio.h>

#include "dzs.h"

int main() {
    int bad = 0;
    const double a[][2] = {{0.02, 0.0216}, {0.5, 0.55}, {0.9247, 1.0}, {0.1, 0.1001}};
    for (const auto &s : a) {
        dzs_step_params p{};
        bad += dzs_step_factors(s[0], s[1], 0.3, &p) != DZS_OK;
        bad += !(p.K1 > 0.0 && p.K2 > 0.0 && p.lc.D > 0.0 && p.lc.n_cheb >= 1);
    }
    dzs_step_params q{};
    bad += dzs_step_factors(0.5, 0.4, 0.3, &q) == DZS_OK;      // a1 < a0
    bad += dzs_step_factors(0.5, 1.2, 0.3, &q) == DZS_OK;      // past a = 1
    bad += dzs_step_factors(0.5, 0.6, 0.3, nullptr) == DZS_OK;
    dzs_halt_params hp{1.1, 0.5, 100.0, 50.0};
    dzs_halt_state hs{1.2, 0.4, 0.6, 120.0, 60.0};
    const unsigned r = dzs_halt_check(&hp, &hs);
    bad += (r & DZS_HALT_BALANCE) == 0 || (r & DZS_HALT_RATIO) == 0;
    bad += dzs_halt_check(nullptr, &hs) != 0;
    dzs_forecast f{};
    bad += dzs_forecast_speedup(4000.0, 4e12, 0.3, &f) != DZS_OK || !(f.speedup > 1.0);
    bad += dzs_forecast_speedup(-1.0, 4e12, 0.3, &f) == DZS_OK;
    bad += dzs_forecast_speedup(4000.0, 4e12, 0.3, nullptr) == DZS_OK;
    printf("host ABI driver: %d unexpected results, forecast %g\n", bad, f.speedup);
    return bad == 0 ? 0 : 1;
}

// Host-side checks of libwcirc under AddressSanitizer (CPU only, no device call): status
// strings, option defaults, plan footprints over a grid of valid and invalid problems
// (the validation and sizing code), and plan creation refused before any device work.
#include <cstdio>
#include <cmath>
#include "wc.h"
int main() {
  int bad = 0;
  for (int c = -1; c < 14; ++c) if (!wc_status_str(c)) ++bad;
  std::printf("%s\n", wc_version());
  wc_opts o; wc_opts_default(&o);
  double af[2 * 7 * 8];
  for (double &a : af) a = 1.0;
  for (int dims = 0; dims <= 3; ++dims)
    for (int M : {0, 1, 2, 7, 31, 32, 1023})
      for (int n : {1, 2, 3, 16, 1024})
        for (int method = -1; method <= 3; ++method)
          for (int disc = 0; disc <= 2; ++disc)
            for (int bc = 0; bc <= 2; ++bc)
              for (int lr = 0; lr <= 1; ++lr) {
                wc_problem p{};
                p.dims = dims; p.M = M; p.n = n; p.T = 1; p.theta = 0.5; p.gamma = 1e-4;
                p.zeta = M_PI; p.s2_remedy = 1; p.disc = disc; p.bc = bc; p.kappa = 1;
                p.a_face_host = (M == 7 && dims == 2 && disc == 0) ? af : nullptr;
                o.method = method; o.lowrank = lr;
                (void)wc_plan_footprint_bytes(&p, &o);
                wc_plan *pl = nullptr;
                if (dims == 0 || M == 0) {  // invalid: refused before any device call
                  if (wc_plan_create(&p, &o, nullptr, &pl) == WC_OK || pl) ++bad;
                }
              }
  std::printf("bad %d\n", bad);
  return bad;
}

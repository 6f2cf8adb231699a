// Host driver for the sanitizer build of the pre-factorisation (plan.cpp):
// builds plans over a grid of shapes -- r, n (tiny, ragged, powers of two,
// long), partition counts (1, powers of two and not), cyclic and acyclic,
// per-row bands, precisions, rows per lane and interior solves -- so that
// AddressSanitizer and UndefinedBehaviorSanitizer see every index path of the
// host code.  Prints the number of plans built and rejected; exits non-zero
// only through a sanitizer report.
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "../paper_2101_02286_amd/csrc/plan.h"

int main() {
  int built = 0, rejected = 0;
  std::mt19937 rng(7);
  std::uniform_real_distribution<double> u(-0.3, 0.3);
  const int ns[] = {3, 5, 8, 11, 37, 64, 100, 256, 384, 613, 1024, 4100};
  const int Ps[] = {0, 1, 2, 3, 5, 8, 16};
  const int rpls[] = {0, 4, 6, 8, 12, 16, 32};
  for (int r = 1; r <= 2; ++r)
    for (int n : ns)
      for (int P : Ps)
        for (int cyclic = 0; cyclic <= 1; ++cyclic)
          for (int per_row = 0; per_row <= 1; ++per_row)
            for (int prec = 0; prec <= 2; ++prec)
              for (int rpl : rpls)
                for (int interior = 0; interior <= 2; ++interior) {
                  // keep the grid bounded: the expensive combinations once
                  if (n >= 1024 && (per_row || prec == 1 || (rpl != 0 && rpl != 16) || interior == 1)) continue;
                  if (prec == 1) continue;  // plain FP32 takes FP32 + refinement's layouts
                  if (interior == 1 && rpl != 0 && rpl != 8) continue;
                  if (P > 1 && (rpl == 4 || rpl == 6 || rpl == 12 || rpl == 32)) continue;
                  const int w = 2 * r + 1;
                  std::vector<double> bands(per_row ? (size_t)n * w : (size_t)w);
                  for (size_t i = 0; i < bands.size(); ++i) {
                    const int o = (int)(i % w) - r;
                    bands[i] = o == 0 ? 1.0 : (per_row ? u(rng) : (r == 1 ? 1.0 / 3 : (o == 1 || o == -1 ? 0.5 : 0.05)));
                  }
                  cb_plan_desc d{};
                  d.r = r;
                  d.n = n;
                  d.bands = bands.data();
                  d.per_row = per_row;
                  d.cyclic = cyclic;
                  d.partitions = P;
                  d.precision = prec;
                  d.rows_per_lane = rpl;
                  d.interior = interior;
                  d.host_only = 1;
                  cb::Plan p;
                  std::string msg;
                  if (cb::build_plan(d, p, msg) == CB_OK) ++built;
                  else ++rejected;
                }
  std::printf("plans built %d rejected %d\n", built, rejected);
  return built > 0 ? 0 : 1;
}

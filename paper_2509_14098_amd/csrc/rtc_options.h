// Compile options of the generated sweep programs (used by the qsv_rtc helper;
// the library hashes them into the code-object cache key).  Packed FP32
// instructions stay disabled, as in the library's own build.  Amplitudes,
// matrices and their products are finite and the sign of a zero amplitude
// does not matter, so the compiler may drop multiplications by the exact
// zeros and ones of a partition's constant matrices.
#pragma once

namespace qsv {
static const char *const rtc_options[] = {"--offload-arch=gfx950", "-O3", "-std=c++17",
                                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                                          "-ffinite-math-only", "-fno-signed-zeros"};
constexpr int rtc_n_options = (int)(sizeof rtc_options / sizeof rtc_options[0]);
}  // namespace qsv

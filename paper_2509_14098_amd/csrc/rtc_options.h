// Compile options of the generated sweep programs (used by the qsv_rtc helper;
// the library hashes them into the code-object cache key).  Packed FP32
// instructions stay disabled, as in the library's own build.
#pragma once

namespace qsv {
static const char *const rtc_options[] = {"--offload-arch=gfx950", "-O3", "-std=c++17",
                                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
constexpr int rtc_n_options = (int)(sizeof rtc_options / sizeof rtc_options[0]);
}  // namespace qsv

// qsv_rtc: compiles one generated program of specialised partition sweeps
// (written by specialise_source) for gfx950 with hipRTC.
//
//   qsv_rtc <source.hip> <code object out> <log out>
//
// Exit status 0 on success; otherwise the compiler log is in <log out>.  The
// device headers the programs include are embedded at build time.  The
// helper touches no GPU: it runs as a child process of the library so that
// several programs compile at once (hipRTC serialises compiles within one
// process).
#include <hip/hiprtc.h>

#include <fstream>
#include <iterator>
#include <string>
#include <vector>

#include "rtc_options.h"

namespace qsv {
extern const int rtc_n_headers;
extern const char *const rtc_header_names[];
extern const char *const rtc_header_texts[];
}  // namespace qsv

int main(int argc, char **argv)
{
    if (argc != 4) return 2;
    std::ifstream in(argv[1], std::ios::binary);
    const std::string src((std::istreambuf_iterator<char>(in)), std::istreambuf_iterator<char>());
    std::ofstream log(argv[3], std::ios::binary);
    if (src.empty()) {
        log << "empty source " << argv[1] << "\n";
        return 1;
    }
    hiprtcProgram prog;
    hiprtcResult r = hiprtcCreateProgram(&prog, src.c_str(), argv[1], qsv::rtc_n_headers, qsv::rtc_header_texts,
                                         qsv::rtc_header_names);
    if (r != HIPRTC_SUCCESS) {
        log << "hiprtcCreateProgram: " << hiprtcGetErrorString(r) << "\n";
        return 1;
    }
    r = hiprtcCompileProgram(prog, qsv::rtc_n_options, const_cast<const char **>(qsv::rtc_options));
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    if (n > 1) {
        std::string text(n, '\0');
        hiprtcGetProgramLog(prog, &text[0]);
        log << text;
    }
    if (r != HIPRTC_SUCCESS) {
        log << "hiprtcCompileProgram: " << hiprtcGetErrorString(r) << "\n";
        hiprtcDestroyProgram(&prog);
        return 1;
    }
    hiprtcGetCodeSize(prog, &n);
    std::vector<char> code(n);
    if (n) hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    std::ofstream out(argv[2], std::ios::binary);
    out.write(code.data(), (std::streamsize)code.size());
    return (n > 0 && out) ? 0 : 1;
}

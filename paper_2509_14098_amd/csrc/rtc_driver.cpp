// Compilation of the generated programs of specialised partition sweeps
// (specialise.cpp writes them).  The programs are compiled for gfx950 by the
// helper executable qsv_rtc (hipRTC), which sits beside the library; hipRTC
// serialises compiles within one process, so up to 16 helpers run at once as
// child processes.  The caller loads the code objects.
//
// Code-object cache (optional): with QSV_KERNEL_CACHE=<dir> every program's
// code object is kept in <dir>/<key>.co, the key being a 64-bit FNV-1a hash
// of the program, the embedded device headers and the compile options; a
// later plan with the same program loads it instead of compiling.  With
// QSV_KERNEL_CACHE_ONLY=1 as well, a program missing from the cache is an
// error and no compiler process is started (for runs under a profiler).
#include <dlfcn.h>
#include <spawn.h>
#include <sys/stat.h>
#include <sys/wait.h>
#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <fstream>
#include <functional>
#include <iterator>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "rtc_options.h"

extern char **environ;

namespace qsv {

// The device headers the generated programs include (embedded at build time).
extern const int rtc_n_headers;
extern const char *const rtc_header_names[];
extern const char *const rtc_header_texts[];

namespace {

std::string read_file(const std::string &path)
{
    std::ifstream f(path, std::ios::binary);
    return std::string(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
}

// The helper executable next to this library.
std::string helper_path()
{
    Dl_info info;
    if (!dladdr((void *)&helper_path, &info) || !info.dli_fname) return "qsv_rtc";
    std::string lib = info.dli_fname;
    const size_t slash = lib.rfind('/');
    return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/qsv_rtc";
}

uint64_t fnv1a(uint64_t h, const std::string &s)
{
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

std::string cache_key(const std::string &src)
{
    uint64_t h = 1469598103934665603ull;
    for (int i = 0; i < rtc_n_options; ++i) h = fnv1a(h, rtc_options[i]);
    for (int i = 0; i < rtc_n_headers; ++i) h = fnv1a(fnv1a(h, rtc_header_names[i]), rtc_header_texts[i]);
    h = fnv1a(h, src);
    char b[24];
    std::snprintf(b, sizeof b, "%016llx", (unsigned long long)h);
    return b;
}

struct TempDir {
    std::string path;
    std::vector<std::string> files;
    ~TempDir()
    {
        for (const std::string &f : files) std::remove(f.c_str());
        if (!path.empty()) rmdir(path.c_str());
    }
};

}  // namespace

namespace {

// Compiles the program texts (code objects into codes[i]) in up to nc helper
// processes at a time, through the code-object cache when one is set;
// on_done(i), on the calling thread, as soon as codes[i] is filled.  Returns ""
// or the first error (with the compiler log); labels name the programs in it.
std::string compile_texts(const std::vector<std::string> &texts, const std::vector<std::string> &labels,
                          std::vector<std::vector<char>> &codes, int nc, const std::function<void(size_t)> &on_done)
{
    const size_t n = texts.size();
    codes.assign(n, {});
    const std::string helper = helper_path();
    TempDir tmp;
    const char *td = std::getenv("TMPDIR");
    std::string tmpl = std::string(td && *td ? td : "/tmp") + "/qsv_rtc_XXXXXX";
    std::vector<char> tb(tmpl.begin(), tmpl.end());
    tb.push_back('\0');
    if (!mkdtemp(tb.data())) return "cannot create a temporary directory for the generated kernels";
    tmp.path = tb.data();
    const char *cdir = std::getenv("QSV_KERNEL_CACHE");
    const std::string cache = cdir && *cdir ? cdir : "";
    const char *conly = std::getenv("QSV_KERNEL_CACHE_ONLY");
    const bool cache_only = !cache.empty() && conly && *conly && std::string(conly) != "0";
    if (!cache.empty() && !cache_only) (void)mkdir(cache.c_str(), 0777);  // the cache directory itself, if missing
    std::vector<std::string> src(n), out(n), log(n), cached(n);
    std::vector<size_t> todo;
    for (size_t c = 0; c < n; ++c) {
        if (!cache.empty()) {
            cached[c] = cache + "/" + cache_key(texts[c]) + ".co";
            const std::string code = read_file(cached[c]);
            if (!code.empty()) {
                codes[c].assign(code.begin(), code.end());
                if (on_done) on_done(c);
                continue;
            }
            if (cache_only) return "kernel not in the cache (QSV_KERNEL_CACHE_ONLY is set): " + cached[c];
        }
        src[c] = tmp.path + "/p" + std::to_string(c) + ".hip";
        out[c] = tmp.path + "/p" + std::to_string(c) + ".co";
        log[c] = tmp.path + "/p" + std::to_string(c) + ".log";
        tmp.files.insert(tmp.files.end(), {src[c], out[c], log[c]});
        std::ofstream f(src[c], std::ios::binary);
        f << texts[c];
        if (!f) return "cannot write " + src[c];
        todo.push_back(c);
    }
    if (!todo.empty() && access(helper.c_str(), X_OK) != 0) return "compiler helper not found: " + helper;
    // run the helpers, at most nc at a time; wait only for our own children
    std::string err;
    std::vector<pid_t> pid(n, -1);
    std::deque<size_t> running;
    size_t next = 0;
    for (;;) {
        while (err.empty() && next < todo.size() && (int)running.size() < nc) {
            const size_t c = todo[next++];
            std::string a0 = helper;
            char *argv[] = {&a0[0], &src[c][0], &out[c][0], &log[c][0], nullptr};
            pid_t child;
            if (posix_spawn(&child, helper.c_str(), nullptr, nullptr, argv, environ) != 0) {
                err = "cannot start " + helper;
                break;
            }
            pid[c] = child;
            running.push_back(c);
        }
        if (running.empty()) break;
        const size_t c = running.front();
        running.pop_front();
        int st = 0;
        pid_t w;
        do w = waitpid(pid[c], &st, 0);  // a signal to the host process must not orphan the child
        while (w < 0 && errno == EINTR);
        if (w != pid[c]) {
            if (err.empty()) err = "waitpid failed";
            continue;
        }
        if (!(WIFEXITED(st) && WEXITSTATUS(st) == 0) && err.empty()) {
            std::string l = read_file(log[c]);
            if (l.size() > 4000) l.resize(4000);
            err = "kernel compile failed for " + labels[c] + ": " + l;
        }
        if (!err.empty()) continue;
        const std::string code = read_file(out[c]);
        if (code.empty()) {
            err = "no code object from the compiler helper for " + labels[c];
            continue;
        }
        codes[c].assign(code.begin(), code.end());
        if (!cached[c].empty()) {  // publish by rename, so readers see whole files only
            const std::string part = cached[c] + "." + std::to_string(getpid()) + ".tmp";
            std::ofstream f(part, std::ios::binary);
            f.write(code.data(), (std::streamsize)code.size());
            f.close();
            if (!f || std::rename(part.c_str(), cached[c].c_str()) != 0) std::remove(part.c_str());
        }
        if (on_done) on_done(c);
    }
    return err;
}

}  // namespace

std::string specialise_compile(const Plan &plan, std::vector<SpecChunk> &chunks, int max_procs,
                               const std::vector<int> *subset, int chunk_partitions,
                               const std::function<void(size_t)> &on_chunk,
                               const std::function<void(size_t)> &on_sized)
{
    const int np = (int)plan.parts.size();
    chunks.clear();
    if (np == 0) return "";
    const bool with_reverse = !subset && specialise_reverse(plan);
    unsigned hw = std::thread::hardware_concurrency();
    const int nc = std::max(1, std::min({np, max_procs, hw ? (int)hw : 1}));
    // contiguous partition ranges of near-equal op counts
    std::vector<int64_t> cum(np + 1, 0);
    for (int p = 0; p < np; ++p) {
        const DevPart &P = plan.parts[p];
        int64_t n = 1;
        for (int s = P.stage_begin; s < P.stage_end; ++s) n += plan.stages[s].op_end - plan.stages[s].op_begin;
        cum[p + 1] = cum[p] + n;
    }
    int p = 0;
    if (subset) {  // one program per listed partition
        for (int q : *subset) {
            SpecChunk ch;
            ch.p0 = q;
            ch.p1 = q + 1;
            chunks.push_back(ch);
        }
        p = np;
    }
    if (chunk_partitions > 0) {
        // chunk_partitions per program, the last partitions first: an apply that
        // starts while they compile reaches the late partitions last
        for (int q = np; q > 0; q -= chunk_partitions) {
            SpecChunk ch;
            ch.p0 = std::max(0, q - chunk_partitions);
            ch.p1 = q;
            chunks.push_back(ch);
        }
        p = np;
    }
    for (int c = 0; c < nc && p < np; ++c) {
        SpecChunk ch;
        ch.p0 = p;
        const int64_t target = cum[np] * (c + 1) / nc;
        do ++p;
        while (p < np && cum[p + 1] <= target);
        if (c == nc - 1) p = np;
        ch.p1 = p;
        chunks.push_back(ch);
    }
    if (on_sized) on_sized(chunks.size());
    std::vector<std::string> texts, labels;
    for (const SpecChunk &ch : chunks) {
        texts.push_back(specialise_source(plan, ch.p0, ch.p1, with_reverse));
        labels.push_back("partitions " + std::to_string(ch.p0) + ".." + std::to_string(ch.p1 - 1));
    }
    std::vector<std::vector<char>> codes;
    return compile_texts(texts, labels, codes, nc, [&](size_t c) {
        chunks[c].code = std::move(codes[c]);
        if (on_chunk) on_chunk(c);
    });
}

std::string specialise_batched_compile(const Plan &plan, std::vector<char> &code)
{
    std::vector<std::vector<char>> codes;
    const std::string err = compile_texts({specialise_batched_source(plan)}, {"the batched kernel"}, codes, 1, nullptr);
    if (err.empty()) code = std::move(codes[0]);
    return err;
}

}  // namespace qsv

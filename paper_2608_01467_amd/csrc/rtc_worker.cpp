// rtc_worker.cpp -- fhs_rtc: compile one consumer source to a gfx950 code
// object with hipRTC (the same options as the library's run-time
// compilation).  hipRTC serialises compilations inside a process, so
// fhs_precompile runs several of these as child processes to compile many
// splits at once.  No HIP runtime call is made: the process never touches
// the GPU.
//
//   fhs_rtc <source file> <code object out> <log out>
//
// Exit status 0 on success, 1 if the compilation fails (log written), 2 on
// I/O errors.
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "jit.hpp"

int main(int argc, char **argv) {
    if (argc != 4) {
        std::fprintf(stderr, "usage: fhs_rtc <source> <code out> <log out>\n");
        return 2;
    }
    std::ifstream in(argv[1], std::ios::binary);
    if (!in) return 2;
    std::stringstream ss;
    ss << in.rdbuf();
    std::vector<char> code;
    std::string log;
    const bool ok = fhs::compile_code(ss.str(), code, log);
    std::ofstream lg(argv[3], std::ios::binary);
    lg << log;
    if (!ok) return 1;
    std::ofstream out(argv[2], std::ios::binary);
    out.write(code.data(), static_cast<std::streamsize>(code.size()));
    return out ? 0 : 2;
}

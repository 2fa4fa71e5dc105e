// Host build of the step kernel's FP64 elementary functions: reads n
// doubles per function from argv[1] (exp, log, log1p, sincospi and
// reciprocal/square-root arguments, n each) and writes exp, log, log1p,
// sin(pi x), cos(pi x), 1/x, sqrt(x), and the forms without special cases
// exp_fin (of the exp arguments) and log1p_fin (of the log1p arguments) to
// argv[2].
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "gccd_fp64.h"

int main(int argc, char** argv) {
    if (argc != 4) return 2;
    const long n = std::atol(argv[3]);
    std::vector<double> in(5 * n), out(9 * n);
    FILE* f = std::fopen(argv[1], "rb");
    if (!f || std::fread(in.data(), sizeof(double), in.size(), f) != in.size()) return 3;
    std::fclose(f);
    for (long i = 0; i < n; ++i) {
        out[i] = gccd::fp64::exp(in[i]);
        out[n + i] = gccd::fp64::log(in[n + i]);
        out[2 * n + i] = gccd::fp64::log1p(in[2 * n + i]);
        gccd::fp64::sincospi(in[3 * n + i], &out[3 * n + i], &out[4 * n + i]);
        out[5 * n + i] = gccd::fp64::recip(in[4 * n + i]);
        out[6 * n + i] = gccd::fp64::sqrt_pos(in[4 * n + i]);
        out[7 * n + i] = gccd::fp64::exp_fin(in[i]);
        out[8 * n + i] = gccd::fp64::log1p_fin(in[2 * n + i]);
    }
    f = std::fopen(argv[2], "wb");
    if (!f || std::fwrite(out.data(), sizeof(double), out.size(), f) != out.size()) return 4;
    std::fclose(f);
    return 0;
}

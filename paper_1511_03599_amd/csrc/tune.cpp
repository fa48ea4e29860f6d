// Tuning cache: a small text file, one entry per line,
//   <arch> <dtype> <C> <T> <B> <S> path=<p> fir_cpt=<n> fir_sb=<n> fused_sb=<n> chunk_mib=<n>
// Lines that do not parse are ignored, so a damaged cache degrades to the
// built-in defaults rather than to an error.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "tune.h"

namespace pfb {

std::string device_arch_name()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return "unknown";
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

static bool parse_kv(const char *tok, const char *key, int *val)
{
    const size_t n = std::strlen(key);
    if (std::strncmp(tok, key, n) != 0 || tok[n] != '=')
        return false;
    char *end = nullptr;
    long v = std::strtol(tok + n + 1, &end, 10);
    if (end == tok + n + 1)
        return false;
    *val = (int)v;
    return true;
}

bool tune_lookup(const pfb_desc &d, TuneEntry *out)
{
    const char *path = std::getenv("PFB_TUNE_CACHE");
    if (!path || !*path)
        return false;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return false;
    const std::string arch = device_arch_name();
    char line[512];
    bool found = false;
    TuneEntry best;
    while (std::fgets(line, sizeof line, f)) {
        char a[64];
        int dt, C, T, B;
        long long S;
        int used = 0;
        if (std::sscanf(line, "%63s %d %d %d %d %lld%n", a, &dt, &C, &T, &B, &S, &used) != 6)
            continue;
        if (arch != a || dt != d.dtype || C != d.channels || T != d.taps || B != d.batch || S != d.spectra)
            continue;
        TuneEntry e;
        char *rest = line + used;
        for (char *tok = std::strtok(rest, " \t\r\n"); tok; tok = std::strtok(nullptr, " \t\r\n")) {
            parse_kv(tok, "path", &e.path);
            parse_kv(tok, "fir_cpt", &e.fir_cpt);
            parse_kv(tok, "fir_sb", &e.fir_sb);
            parse_kv(tok, "fused_sb", &e.fused_sb);
            parse_kv(tok, "chunk_mib", &e.chunk_mib);
        }
        best = e; // the last matching line wins
        found = true;
    }
    std::fclose(f);
    if (found)
        *out = best;
    return found;
}

} // namespace pfb

// Host-only driver of the library's mesh validation and table derivation,
// built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer.
// Reads a mesh description (counts, radius, then the descriptor's arrays in
// order) and prints "ok" or "rejected: <reason>".
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "mpdc_internal.h"

template <typename T> static bool rd(FILE *f, std::vector<T> &v, long n) {
    v.resize((size_t)n);
    return n == 0 || fread(v.data(), sizeof(T), (size_t)n, f) == (size_t)n;
}

int main(int argc, char **argv) {
    if (argc != 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t c[3];
    double radius;
    if (fread(c, 4, 3, f) != 3 || fread(&radius, 8, 1, f) != 1) return 2;
    const long N = c[0], E = c[1], V = c[2];
    std::vector<int32_t> coe, voe, off, eoc, voc, cov, eov;
    std::vector<double> xc, xv, xe, de, le, ac, av, ka, fv;
    bool ok = rd(f, coe, 2 * E) && rd(f, voe, 2 * E) && rd(f, off, N + 1) && rd(f, eoc, 2 * E) &&
              rd(f, voc, 2 * E) && rd(f, cov, 3 * V) && rd(f, eov, 3 * V) && rd(f, xc, 3 * N) &&
              rd(f, xv, 3 * V) && rd(f, xe, 3 * E) && rd(f, de, E) && rd(f, le, E) && rd(f, ac, N) &&
              rd(f, av, V) && rd(f, ka, 3 * V) && rd(f, fv, V);
    fclose(f);
    if (!ok) return 2;
    mpdc_mesh_desc d = {c[0], c[1], c[2], coe.data(), voe.data(), off.data(), eoc.data(), voc.data(),
                        cov.data(), eov.data(), xc.data(), xv.data(), xe.data(), de.data(), le.data(),
                        ac.data(), av.data(), ka.data(), fv.data(), radius};
    std::string err = mpdc::validate_mesh(&d);
    if (err.empty()) {
        mpdc::HostTables t;
        err = mpdc::derive_tables(&d, t);
    }
    if (!err.empty()) {
        printf("rejected: %s\n", err.c_str());
        return 3;
    }
    printf("ok\n");
    return 0;
}

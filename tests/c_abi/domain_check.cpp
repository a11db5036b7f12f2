// The host domain builder (saamg_domain_from_shape, multithreaded) built alone with a
// sanitizer and run over the three pipe shapes, closed and open ends, including a box large
// enough to use every worker thread.  Prints one line per case: nodes, unknowns, wall
// entries and a checksum of the fractions; exits non-zero on any error.  The test compares
// the lines with the library's own builder.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "saamg.h"

int main() {
    struct Case {
        int kind;
        double a, b, len, bore, cav;
        int nx, ny, nz, open;
    };
    const Case cases[] = {
        {SAAMG_SHAPE_CYLINDER, 1.0, 1.0, 2.0, 0.0, 0.0, 33, 33, 33, 0},
        {SAAMG_SHAPE_ELLIPSE, 1.0, 0.6, 4.0, 0.0, 0.0, 70, 45, 66, 0},
        {SAAMG_SHAPE_BOXBORE, 0.8, 0.8, 4.0, 0.5, 4.0 / 6.0, 41, 41, 83, 0},
        {SAAMG_SHAPE_CYLINDER, 1.0, 1.0, 2.0, 0.0, 0.0, 27, 27, 25, 1},
        {SAAMG_SHAPE_ELLIPSE, 1.0, 0.6, 4.0, 0.0, 0.0, 96, 96, 160, 0},
    };
    for (const Case& c : cases) {
        const int nzb = c.nz + 2 * c.open;
        const size_t nbox = (size_t)c.nx * c.ny * nzb;
        std::vector<uint8_t> mask(nbox);
        int64_t nw = 0;
        double h[4];
        int rc = saamg_domain_from_shape(c.kind, c.a, c.b, c.len, c.bore, c.cav, c.nx, c.ny, c.nz,
                                         c.open, mask.data(), 0, nullptr, nullptr, nullptr, &nw, h);
        if (rc != SAAMG_OK) return 1;
        std::vector<int64_t> node(nw + 1);
        std::vector<uint8_t> dir(nw + 1);
        std::vector<double> s(nw + 1);
        rc = saamg_domain_from_shape(c.kind, c.a, c.b, c.len, c.bore, c.cav, c.nx, c.ny, c.nz,
                                     c.open, mask.data(), nw, node.data(), dir.data(), s.data(), &nw,
                                     h);
        if (rc != SAAMG_OK) return 1;
        long unk = 0;
        for (uint8_t m : mask) unk += m != 0;
        double sum = 0.0;
        for (int64_t e = 0; e < nw; ++e) sum += s[e] * (double)(1 + dir[e]) + 1e-9 * (double)node[e];
        std::printf("%zu %ld %lld %.12e\n", nbox, unk, (long long)nw, sum);
    }
    return 0;
}

// The host-side domain preparation of the setup (saamg::prepare_domain, multithreaded:
// checks of the mask and the wall entries, the near-wall rows and their six wall fractions)
// built alone with a sanitizer, on domains from the host domain builder.  Per case and
// boundary variant one line: "ok <rows> <sum of row nodes> <checksum of the fractions>",
// or "err <message>" for the invalid domains.  The test recomputes the rows from the
// builder's output with numpy.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_0907_4863_amd/csrc/host_prep.h"

static void run(const saamg_domain& d, int variant) {
    try {
        const saamg::DomainPrep D = saamg::prepare_domain(&d, variant);
        long long sn = 0;
        double cs = 0.0;
        for (size_t r = 0; r < D.nw_nodes.size(); ++r) {
            sn += (long long)D.nw_nodes.data()[r];
            for (int q = 0; q < 6; ++q) cs += D.nw_frac.data()[6 * r + q] * (double)(1 + q);
        }
        std::printf("ok %zu %lld %.15e\n", D.nw_nodes.size(), sn, cs);
    } catch (const saamg::ApiError& e) {
        std::printf("err %s\n", e.msg.c_str());
    }
}

int main() {
    struct Case {
        int kind;
        double a, b, len, bore, cav;
        int nx, ny, nz, open;
    };
    const Case cases[] = {
        {SAAMG_SHAPE_CYLINDER, 1.0, 1.0, 2.0, 0.0, 0.0, 33, 33, 33, 0},
        {SAAMG_SHAPE_BOXBORE, 0.8, 0.8, 4.0, 0.5, 4.0 / 6.0, 41, 41, 83, 0},
        {SAAMG_SHAPE_CYLINDER, 1.0, 1.0, 2.0, 0.0, 0.0, 27, 27, 25, 1},
        {SAAMG_SHAPE_ELLIPSE, 1.0, 0.6, 4.0, 0.0, 0.0, 96, 96, 160, 0},
        {SAAMG_SHAPE_ELLIPSE, 1.0, 0.6, 4.0, 0.0, 0.0, 128, 128, 200, 1},
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
        const saamg_domain d{c.nx, c.ny, nzb, h[0], h[1], h[2], mask.data(), nw, node.data(),
                             dir.data(), s.data(), h[3]};
        for (int v = SAAMG_VARIANT_CONST; v <= SAAMG_VARIANT_QUAD; ++v) run(d, v);
        // the same entries in a shuffled order
        std::vector<int64_t> perm(nw);
        for (int64_t e = 0; e < nw; ++e) perm[e] = e;
        std::shuffle(perm.begin(), perm.end(), std::mt19937_64(12345));
        std::vector<int64_t> node2(nw + 1);
        std::vector<uint8_t> dir2(nw + 1);
        std::vector<double> s2(nw + 1);
        for (int64_t e = 0; e < nw; ++e) {
            node2[e] = node[perm[e]];
            dir2[e] = dir[perm[e]];
            s2[e] = s[perm[e]];
        }
        saamg_domain d2 = d;
        d2.wall_node = node2.data();
        d2.wall_dir = dir2.data();
        d2.wall_s = s2.data();
        run(d2, SAAMG_VARIANT_QUAD);
        // invalid domains: a duplicated entry, a fraction of 0, a node out of range (each
        // near the end of the entries, after a valid half), an unknown on a face
        saamg_domain e = d2;
        e.n_wall = nw + 1;
        node2[nw] = node2[nw / 2];
        dir2[nw] = dir2[nw / 2];
        s2[nw] = s2[nw / 2];
        run(e, SAAMG_VARIANT_QUAD);
        const double keep_s = s2[nw - 2];
        s2[nw - 2] = 0.0;
        run(d2, SAAMG_VARIANT_QUAD);
        s2[nw - 2] = keep_s;
        const int64_t keep_n = node2[nw - 3];
        node2[nw - 3] = -1;
        run(d2, SAAMG_VARIANT_QUAD);
        node2[nw - 3] = keep_n;
        std::vector<uint8_t> m2 = mask;
        m2[(size_t)c.nx * c.ny * (nzb / 2) + (size_t)c.nx * (c.ny / 2)] = 1;  // x = 0
        saamg_domain f = d;
        f.mask = m2.data();
        run(f, SAAMG_VARIANT_QUAD);
    }
    return 0;
}

// Host-side preparation of a discrete domain for the setup: argument checks and the
// near-wall rows (Section 2: the unknowns next to the wall and their wall fractions).
// Plain C++ with no HIP dependency, so that it can also be built and checked on its own.
#pragma once

#include <cstddef>
#include <cstdint>
#include <memory>
#include <string>

#include "../../include/saamg.h"

namespace saamg {

// An error of an entry point: a status code of the C interface and its message.
struct ApiError {
    int status;
    std::string msg;
};

// Host array left uninitialised by the allocation (the threads that fill it touch its
// pages first).
template <class T>
struct HostArr {
    std::unique_ptr<T[]> p;
    size_t n = 0;
    void alloc(size_t m) {
        p.reset(m ? new T[m] : nullptr);
        n = m;
    }
    size_t size() const { return n; }
    bool empty() const { return n == 0; }
    const T* data() const { return p.get(); }
    T& operator[](size_t i) { return p[i]; }
};

// Host-side checks of a domain and its near-wall rows: wall fractions below 1 (the
// constant rule ignores them) and, with open ends, every end-plane unknown; six fractions
// per row, 1 where no wall is cut.  The passes over the mask and the wall entries run on
// up to 16 threads; errors are those of the first offending entry in order.
struct DomainPrep {
    HostArr<int64_t> nw_nodes;
    HostArr<double> nw_frac;
};

// scan_mask = false skips the mask's own checks (count, faces, open ends): a refresh
// compares the mask with the hierarchy's, which passed them.  Throws ApiError
// (SAAMG_INVALID_ARG) for an invalid domain.
DomainPrep prepare_domain(const saamg_domain* dom, int variant, bool scan_mask = true);

}  // namespace saamg

// hilbert_order.hip -- host side of the Hilbert order of the super-boxes:
// the orientation tables of the curve, derived once from Skilling's
// transform (AIP Conf. Proc. 707, 2004).
#include "hilbert_order.h"

#include <array>
#include <vector>

namespace abm {
namespace {

// Index of cell c (3 coordinates below 2^bits) on the curve.  The transform,
// top bit level first: for every coordinate in turn, if its bit is set the
// lower bits of the first coordinate are inverted, otherwise the lower bits
// of the two are swapped; then the coordinates are Gray-encoded, and the
// index takes one bit of each per level, the first coordinate's highest.
uint64_t curve_index(std::array<uint32_t, 3> c, int bits) {
    if (bits <= 0) return 0;
    const uint32_t top = 1u << (bits - 1);
    for (uint32_t q = top; q > 1u; q >>= 1) {
        const uint32_t low = q - 1u;
        for (uint32_t& v : c) {
            if (v & q) {
                c[0] ^= low;
            } else {
                const uint32_t diff = (c[0] ^ v) & low;
                c[0] ^= diff;
                v ^= diff;
            }
        }
    }
    c[1] ^= c[0];
    c[2] ^= c[1];
    uint32_t flip = 0;
    for (uint32_t q = top; q > 1u; q >>= 1)
        if (c[2] & q) flip ^= q - 1u;
    uint64_t idx = 0;
    for (int b = bits - 1; b >= 0; --b)
        for (int a = 0; a < 3; ++a) idx = (idx << 1) | (((c[a] ^ flip) >> b) & 1u);
    return idx;
}

using Digits = std::array<uint8_t, 8>;   // per child (x | y << 1 | z << 2): its position among the 8

// Visiting order of the children of the node at depth d with coordinates n
// (2^d nodes per axis): each child's last index digit on the curve at depth d + 1.
Digits child_digits(int d, uint32_t nx, uint32_t ny, uint32_t nz) {
    Digits p{};
    for (uint32_t k = 0; k < 8u; ++k)
        p[k] = uint8_t(curve_index({2u * nx + (k & 1u), 2u * ny + ((k >> 1) & 1u), 2u * nz + (k >> 2)}, d + 1) & 7u);
    return p;
}

}  // namespace

bool build_hilbert_tables(HilbertTables* t) {
    // Orientation states are the distinct child orders met on the curve
    // over 2^6 cells per axis; transitions are read off every node of depth
    // up to 4 (the curve is self-similar, so a few levels meet every state).
    constexpr int kDepth = 6;
    std::vector<Digits> states;
    std::vector<std::array<int, 8>> trans;
    auto state_of = [&](const Digits& p) -> int {
        for (size_t s = 0; s < states.size(); ++s)
            if (states[s] == p) return int(s);
        states.push_back(p);
        std::array<int, 8> none;
        none.fill(-1);
        trans.push_back(none);
        return int(states.size()) - 1;
    };
    state_of(child_digits(0, 0, 0, 0));   // the root: state 0
    for (int d = 0; d + 2 < kDepth; ++d) {
        const uint32_t side = 1u << d;
        for (uint32_t nz = 0; nz < side; ++nz)
            for (uint32_t ny = 0; ny < side; ++ny)
                for (uint32_t nx = 0; nx < side; ++nx) {
                    const int s = state_of(child_digits(d, nx, ny, nz));
                    for (uint32_t k = 0; k < 8u; ++k) {
                        const int c = state_of(child_digits(d + 1, 2u * nx + (k & 1u), 2u * ny + ((k >> 1) & 1u),
                                                            2u * nz + (k >> 2)));
                        if (trans[size_t(s)][k] < 0)
                            trans[size_t(s)][k] = c;
                        else if (trans[size_t(s)][k] != c)
                            return false;
                    }
                }
    }
    if (states.size() > size_t(kHilMaxStates)) return false;
    for (size_t s = 0; s < states.size(); ++s) {
        uint32_t seen = 0;
        for (int k = 0; k < 8; ++k) {
            if (trans[s][k] < 0) return false;   // a state whose transitions were never met
            seen |= 1u << states[s][k];
        }
        if (seen != 0xFFu) return false;         // not an order of the 8 children
    }
    for (int s = 0; s < kHilMaxStates; ++s)
        for (int k = 0; k < 8; ++k) {
            uint8_t m = 0;
            if (size_t(s) < states.size())
                for (int j = 0; j < 8; ++j) m |= uint8_t(states[size_t(s)][j] < states[size_t(s)][k] ? 1u << j : 0u);
            t->before[s * 8 + k] = m;
            t->next[s * 8 + k] = uint8_t(size_t(s) < states.size() ? trans[size_t(s)][k] : 0);
        }
    return true;
}

}  // namespace abm

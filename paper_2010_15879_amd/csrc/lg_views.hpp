// Device views of a packed or plain graph: plain structs of pointers and
// sizes, passed to kernels by value.
#pragma once

#include <cstdint>

namespace lg {

// Elias-Fano offsets: x_v = ((select1(H, v) - v) << l) | L[v].
struct EFView {
    const uint64_t *L;        // low bits, l per value
    const uint64_t *H;        // upper bit vector
    const uint32_t *rank_sb;  // rank1(512 b)
    const uint32_t *sel;      // select1(64 j)
    uint32_t l;
    uint32_t n_sel;           // entries of sel
    uint32_t n_sb;            // superblocks = entries of rank_sb - 1
    uint32_t n_hw;            // words of H
};

// Interleaved bit vector (bvIL): block j at words [9j, 9j + 9): the number of
// ones before it, then 512 bits of the vector whose one for list v sits at
// x_v + v.
struct ILView {
    const uint64_t *W;
    uint64_t blocks;
};

// Packed offsets: value v at bits [v*w, v*w + w).
struct POffView {
    const uint64_t *O;
    uint32_t w;
};

struct PackedView {
    const uint32_t *A32;      // packed lists viewed as 32-bit words
    const uint64_t *W;        // width table (local modes)
    const uint64_t *G;        // gap-width table (gap mode)
    uint32_t s;               // global width
    uint32_t F;               // width field bits
    POffView po;
    EFView ef;
    ILView il;
};

struct PlainView {
    const void *off;          // uint32 or uint64 offsets
    const uint32_t *col;
};

}  // namespace lg

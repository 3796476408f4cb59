/* Reference Huffman decoder: a plain binary-tree walk, one bit at a time.
 *
 * Test infrastructure only (see oracle/__init__.py).  The paper reads its
 * Huffman tree top-down, a 0 bit taking the left branch and a 1 bit the right
 * one, until a leaf holds the decoded symbol (section 4.1, Fig. 3).  The tree
 * itself is built on the Python side from (symbol, code, length) triples.
 *
 * Bits are MSB-first inside 32-bit words.
 */
#include <stdint.h>

/* Decode nsym symbols starting at absolute bit position start_bit.
 * left/right: child node ids (-1 when absent), leaf: symbol id or -1.
 * Returns the bit position after the last symbol, or -1 on an invalid path
 * (missing child) or a read past nwords. */
int64_t walk_decode(const int32_t *left, const int32_t *right, const int32_t *leaf,
                    const uint32_t *words, int64_t nwords, int64_t start_bit,
                    int64_t nsym, int32_t *out)
{
    int64_t bit = start_bit;
    for (int64_t i = 0; i < nsym; ++i) {
        int32_t node = 0;
        while (leaf[node] < 0) {
            int64_t w = bit >> 5;
            if (w >= nwords) return -1;
            uint32_t b = (words[w] >> (31 - (bit & 31))) & 1u;
            node = b ? right[node] : left[node];
            ++bit;
            if (node < 0) return -1;
        }
        out[i] = leaf[node];
    }
    return bit;
}

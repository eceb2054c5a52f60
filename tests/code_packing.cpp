// Exhaustive host check of the 16-bit stencil-code packing (codes.h): every
// component field the neighbourhood evaluation can produce, every packed value.
#include "codes.h"

#include <cstdio>

using namespace ps;

static const uint32_t kStencil[6] = {0, 1, 2, 3, 5, 6};  // L | R << 1 | F << 2, F only beside one wall

int main()
{
    // the 37 fields of one component: 36 fluid ones, and solid (its stencil bits ignored)
    uint32_t fields[37];
    int nf = 0;
    for (uint32_t a : kStencil)
        for (uint32_t b : kStencil) fields[nf++] = a | b << 3;
    fields[nf++] = kSolidBit;
    long checked = 0;
    for (int i = 0; i < 37; ++i)
        for (int j = 0; j < 37; ++j)
            for (int k = 0; k < 37; ++k) {
                const uint32_t word = fields[i] | fields[j] << kCodeBits | fields[k] << (2 * kCodeBits);
                const uint32_t p = pack_code(word);
                if (p >= kPackBase * kPackUV || unpack_code(p) != word) {
                    std::printf("round trip failed: word %06x packed %u unpacked %06x\n", word, p, unpack_code(p));
                    return 1;
                }
                // a solid face keeps only its solid bit, whatever stencil bits it carried
                for (uint32_t junk = 1; junk < 64; junk += 9) {
                    uint32_t w2 = word;
                    if (i == 36) w2 |= junk;
                    if (j == 36) w2 |= junk << kCodeBits;
                    if (k == 36) w2 |= junk << (2 * kCodeBits);
                    if (pack_code(w2) != p) {
                        std::printf("solid stencil bits leak: word %06x\n", w2);
                        return 1;
                    }
                }
                ++checked;
            }
    // every packed value is one of the words above
    for (uint32_t p = 0; p < kPackBase * kPackUV; ++p)
        if (pack_code(unpack_code(p)) != p) {
            std::printf("packed value %u does not survive\n", p);
            return 1;
        }
    std::printf("ok %ld\n", checked);
    return 0;
}

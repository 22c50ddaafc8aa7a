// Host-side checks of the index arithmetic the kernels share (compiled for the
// host only from the library's own header):
//   - xcd_block maps the hardware blocks of a launch one-to-one onto its
//     logical blocks, for any block count;
//   - the tiled EO addressing (tile_off) covers every padded slab exactly once
//     for each field's plane list, and blocks_of covers every site;
//   - the LDS reservation of the wave cap leaves room for exactly the wanted
//     number of workgroups per CU on a 160 KiB-LDS CU, whatever the kernel's
//     own LDS (up to 256 B) and for allocation granules of 64 to 1024 bytes.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <vector>

#include "internal.hpp"

static int check_cover(int Vh, size_t sb, const std::vector<std::pair<size_t, size_t>> &planes) {
    const size_t bytes = (size_t)pad_sites(Vh) * sb;
    std::vector<unsigned char> hit(bytes, 0);
    for (int i = 0; i < pad_sites(Vh); i++)
        for (auto &p : planes) {
            const size_t o = tile_off(i, sb, p.first, p.second);
            for (size_t k = 0; k < p.second; k++)
                if (o + k >= bytes || hit[o + k]++) return 1;
        }
    for (size_t k = 0; k < bytes; k++)
        if (hit[k] != 1) return 1;
    return 0;
}

int main() {
    const int nbs[] = {1, 7, 8, 9, 127, 128, 129, 255, 256, 257, 1296, 4096, 20736, 20737, 65537};
    for (int nb : nbs) {
        std::vector<int> seen(nb, 0);
        for (int b = 0; b < nb; b++) {
            const int l = xcd_block(b, nb);
            if (l < 0 || l >= nb || seen[l]++) {
                printf("xcd_block not one-to-one: nb %d b %d -> %d\n", nb, b, l);
                return 1;
            }
        }
    }
    for (int chunk : {-1, 0, 1, 2, 8, 16, 32, 64, 1000}) {
        for (int nb : nbs) {
            std::vector<int> seen(nb, 0);
            for (int b = 0; b < nb; b++) {
                const int l = xcd_block(b, nb, chunk);
                if (l < 0 || l >= nb || seen[l]++) {
                    printf("xcd_block not one-to-one: nb %d chunk %d b %d -> %d\n", nb, chunk, b, l);
                    return 1;
                }
            }
        }
    }
    {
        wc_lattice *lat = new wc_lattice();
        if (wave_cap_for(lat, P64) != 8 || wave_cap_for(lat, P32) != 0 || wave_cap_for(lat, P16) != 0) {
            printf("wave cap defaults wrong\n");
            return 1;
        }
        // tuned per kernel class; a pinned cap and the tuner's forced one take precedence
        lat->cap_tuned[P32][1] = 12;
        lat->cap_tuned[P64][0] = 0;
        if (wave_cap_for(lat, P32, M_DHAT) != 12 || wave_cap_for(lat, P32, M_HOPINV) != 0 ||
            wave_cap_for(lat, P32, M_DFULL) != 0 || wave_cap_for(lat, P64, M_HOPINV) != 0 ||
            wave_cap_for(lat, P64, M_DHAT) != 8) {
            printf("tuned wave caps wrong\n");
            return 1;
        }
        lat->wave_cap[P32] = 4;
        if (wave_cap_for(lat, P32, M_DHAT) != 4) {
            printf("a pinned cap must win over the tuned one\n");
            return 1;
        }
        lat->cap_force = 16;
        if (wave_cap_for(lat, P32, M_DHAT) != 16 || wave_cap_for(lat, P64, M_HOPINV) != 16) {
            printf("the tuner's forced cap must win\n");
            return 1;
        }
        lat->cap_force = -1;
        lat->wave_cap[P32] = -1;
        lat->cap_tuned[P32][1] = lat->cap_tuned[P64][0] = -1;
        for (int lds : {163840}) {
            lat->lds_per_cu = lds;
            for (int cap : {4, 8, 12, 16})
                for (int bs : {64, 128, 256}) {
                    lat->wave_cap[P32] = cap;
                    int want = cap / (bs / 64);
                    if (want < 1) want = 1;
                    const unsigned dyn = cap_lds_bytes(lat, P32, bs);
                    for (unsigned own : {0u, 96u, 256u})
                        for (unsigned gran : {64u, 128u, 256u, 512u, 1024u}) {
                            const unsigned alloc = (dyn + own + gran - 1) / gran * gran;
                            if (dyn == 0 || alloc > (unsigned)lds || (int)(lds / alloc) != want) {
                                printf("wave cap LDS wrong: lds %d cap %d bs %d own %u gran %u: %u bytes -> %u blocks\n",
                                       lds, cap, bs, own, gran, dyn, alloc ? lds / alloc : 0);
                                return 1;
                            }
                        }
                }
            lat->wave_cap[P32] = 0;
            if (cap_lds_bytes(lat, P32, 256) != 0) {
                printf("no cap must reserve nothing\n");
                return 1;
            }
        }
        lat->lds_per_cu = 0;
        if (cap_lds_bytes(lat, P64, 256) != 0) {
            printf("an unknown LDS size must reserve nothing\n");
            return 1;
        }
        delete lat;
    }
    for (int Vh : {1, 63, 64, 65, 1080, 2048, 4097}) {
        for (int bs : {64, 128, 256})
            if ((long)blocks_of(Vh, bs) * bs < Vh || (long)(blocks_of(Vh, bs) - 1) * bs >= Vh) {
                printf("blocks_of wrong: Vh %d bs %d\n", Vh, bs);
                return 1;
            }
        // spinors: FP32 6 x 16 B, FP64 12 x 16 B, FP16 3 x 16 B + 4 B scale
        std::vector<std::pair<size_t, size_t>> s32, s64, s16, l18;
        for (int k = 0; k < 6; k++) s32.push_back({16 * k, 16});
        for (int k = 0; k < 12; k++) s64.push_back({16 * k, 16});
        for (int k = 0; k < 3; k++) s16.push_back({16 * k, 16});
        s16.push_back({48, 4});
        for (int k = 0; k < 4; k++) l18.push_back({16 * k, 16});
        l18.push_back({64, 8});
        if (check_cover(Vh, 96, s32) || check_cover(Vh, 192, s64) || check_cover(Vh, 52, s16) ||
            check_cover(Vh, 72, l18)) {
            printf("tiled addressing does not cover the slab once: Vh %d\n", Vh);
            return 1;
        }
    }
    printf("ok\n");
    return 0;
}

// Runs one CPU variant of the tile pipeline (paper_1209_3332_amd/csrc/host_ops.cpp)
// on an image read from a file, for the sanitizer test: built with
// AddressSanitizer and UBSan, on exact-size allocations and padded pitches, so
// that every access of the host code is checked.
//   driver <op> <conn> <h> <lo> <hi> <height> <width> <in.bin> <out.bin>
// op: 0 h-dome, 1 fill-holes, 2 area filter, 3 markers, 4 labels (int32 out), 5 reconstruction
// by dilation (the input holds the marker plane then the mask plane), 6 distance (int32 out)
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../paper_1209_3332_amd/csrc/host_ops.hpp"

int main(int argc, char **argv) {
    if (argc != 10) return 2;
    const int op = atoi(argv[1]), conn = atoi(argv[2]), h = atoi(argv[3]);
    const long long lo = atoll(argv[4]), hi = atoll(argv[5]);
    const int H = atoi(argv[6]), W = atoi(argv[7]);
    const int planes = op == 5 ? 2 : 1;
    std::vector<unsigned char> in((size_t)H * W * planes);
    FILE *f = fopen(argv[8], "rb");
    if (!f || fread(in.data(), 1, in.size(), f) != in.size()) return 3;
    fclose(f);
    const int64_t pitch = W + 3;   // padded rows; the last row holds exactly W bytes
    auto padded = [&](const unsigned char *src) {
        unsigned char *p = (unsigned char *)malloc((size_t)(H - 1) * pitch + W);
        for (int y = 0; y < H; ++y) memcpy(p + (int64_t)y * pitch, src + (size_t)y * W, W);
        return p;
    };
    hostops::Scratch *s = hostops::scratch_new();
    unsigned char *a = padded(in.data());
    hostops::Plane pa{a, H, W, pitch};
    std::vector<int32_t> out32;
    switch (op) {
        case 0: hostops::hdome(s, pa, h, conn); break;
        case 1: hostops::fill_holes(s, pa, conn); break;
        case 2: hostops::area_threshold(s, pa, conn, lo, hi); break;
        case 3: hostops::pre_watershed(s, pa, conn); break;
        case 4: case 6: {
            const int64_t lp = W + 1;
            int32_t *lab = (int32_t *)malloc(((size_t)(H - 1) * lp + W) * 4);
            if (op == 4) hostops::label(s, pa, lab, lp, conn);
            else hostops::distance2(s, pa, lab, lp);
            out32.resize((size_t)H * W);
            for (int y = 0; y < H; ++y) memcpy(&out32[(size_t)y * W], lab + (int64_t)y * lp, (size_t)W * 4);
            free(lab);
            break;
        }
        case 5: {
            unsigned char *m = padded(in.data() + (size_t)H * W);
            hostops::recon_dilate(s, pa, hostops::Plane{m, H, W, pitch}, conn);
            free(m);
            break;
        }
        default: return 4;
    }
    FILE *o = fopen(argv[9], "wb");
    if (!o) return 5;
    if (!out32.empty()) fwrite(out32.data(), 4, out32.size(), o);
    else
        for (int y = 0; y < H; ++y) fwrite(a + (int64_t)y * pitch, 1, W, o);
    fclose(o);
    free(a);
    hostops::scratch_free(s);
    return 0;
}

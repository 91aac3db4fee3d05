// host_ops.hpp -- CPU variants of the pipeline operations, one host core each.
//
// The paper's runtime runs every operation of a tile's pipeline on either a
// CPU core or a GPU and picks the device per operation instance (Sec. IV-B).
// These are the CPU variants the pipeline scheduler hands to its CPU workers.
// They compute exactly what the GPU operations compute (the results are
// unique, so a tile's bytes do not depend on where each operation ran), with
// algorithms chosen for one core:
//
//  * reconstruction by dilation: a flood in decreasing order of value with one
//    bucket per grey level (each pixel is settled once, at the highest value a
//    path from the marker can bring it: the bottleneck-path form of the
//    reconstruction), O(pixels x neighbours);
//  * labelling: two raster passes with a union-find of provisional labels (the
//    smaller label becomes the root, so a component's root is the label of its
//    first pixel in raster order and numbering the roots in increasing order
//    gives the raster-order numbering);
//  * exact squared Euclidean distance: column distances, then per row the lower
//    envelope of the parabolas (x - i)^2 + g(i)^2 with integer breakpoints.
//
// Every plane is row-major with a pitch in elements >= width.
#pragma once

#include <cstdint>
#include <vector>

namespace hostops {

struct Plane {
    uint8_t *data;
    int height, width;
    int64_t pitch;
    uint8_t *row(int y) const { return data + (int64_t)y * pitch; }
};

struct Scratch;   // per-worker reusable buffers (opaque)
Scratch *scratch_new();
void scratch_free(Scratch *s);

// marker <- rho_mask(min(marker, mask)), in place.
void recon_dilate(Scratch *s, Plane marker, Plane mask, int conn);
// img <- img - rho_img(max(img - h, 0)), in place (h in 1..255).
void hdome(Scratch *s, Plane img, int h, int conn);
// img <- 255 - rho_{255 - img}(frame marker), in place.
void fill_holes(Scratch *s, Plane img, int conn);
// img <- 255 where the 1-dome of img is positive, else 0.
void regional_max(Scratch *s, Plane img, int conn);
// labels <- raster-order component numbers of the nonzero pixels (0 background);
// returns the component count.  labels has label_pitch >= width elements per row.
int32_t label(Scratch *s, Plane img, int32_t *labels, int64_t label_pitch, int conn);
// img <- 255 on components (nonzero pixels, conn) of area in [lo, hi], else 0.
void area_threshold(Scratch *s, Plane img, int conn, int64_t lo, int64_t hi);
// dist2 <- squared distance to the nearest 0 pixel (2^31 - 1 if there is none).
void distance2(Scratch *s, Plane img, int32_t *dist2, int64_t dist_pitch);
// img <- Pre-Watershed markers: regional maxima (conn) of min(floor(sqrt(dist2)), 255).
void pre_watershed(Scratch *s, Plane img, int conn);

}  // namespace hostops

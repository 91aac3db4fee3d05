// host_ops.cpp -- CPU variants of the pipeline operations (see host_ops.hpp).
#include "host_ops.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace hostops {

struct Scratch {
    // padded planes of the flood: one pixel of border around the image, whose
    // mask is 0 so that the border is never raised and needs no bounds checks
    std::vector<uint8_t> val, msk;
    std::vector<uint32_t> bucket[256];
    // labelling
    std::vector<int32_t> prov, parent, count;
    // distance
    std::vector<int32_t> g, s, t;
    std::vector<int32_t> d2;
};

Scratch *scratch_new() { return new Scratch(); }
void scratch_free(Scratch *s) { delete s; }

namespace {

struct Pad {
    int H, W, PW;
    explicit Pad(const Plane &p) : H(p.height), W(p.width), PW(p.width + 2) {}
    size_t size() const { return (size_t)(H + 2) * PW; }
    int64_t at(int y, int x) const { return (int64_t)(y + 1) * PW + (x + 1); }
};

// Flood in decreasing order of value.  On entry s.val holds the clipped marker
// min(J, I) and s.msk the mask, both padded; on exit s.val holds rho_I(J).
// A pixel is settled when its bucket is reached with its current value: no
// path from the marker can bring it higher, since every higher value has been
// settled and passed on to its neighbours already.  Neighbours only receive
// min(value, their mask), which is at most the level being processed, so the
// buckets are visited once each, from 255 down to 1.
void flood(Scratch &s, const Pad &pd, int conn) {
    const int64_t PW = pd.PW;
    const int64_t off[8] = {-1, 1, -PW, PW, -PW - 1, -PW + 1, PW - 1, PW + 1};
    const int nn = conn == 8 ? 8 : 4;
    uint8_t *val = s.val.data();
    const uint8_t *msk = s.msk.data();
    for (int v = 255; v >= 1; --v) {
        std::vector<uint32_t> &b = s.bucket[v];
        while (!b.empty()) {
            const uint32_t p = b.back();
            b.pop_back();
            if (val[p] != (uint8_t)v) continue;   // raised later and settled from a higher bucket
            for (int k = 0; k < nn; ++k) {
                const int64_t q = (int64_t)p + off[k];
                const uint8_t c = std::min<uint8_t>((uint8_t)v, msk[q]);
                if (c > val[q]) {
                    val[q] = c;
                    s.bucket[c].push_back((uint32_t)q);
                }
            }
        }
    }
}

void prepare(Scratch &s, const Pad &pd) {
    s.val.assign(pd.size(), 0);
    s.msk.assign(pd.size(), 0);
    for (auto &b : s.bucket) b.clear();
}

// seed every interior pixel with a nonzero value
void seed_all(Scratch &s, const Pad &pd) {
    for (int y = 0; y < pd.H; ++y) {
        const int64_t r = pd.at(y, 0);
        for (int x = 0; x < pd.W; ++x) {
            const uint8_t v = s.val[r + x];
            if (v) s.bucket[v].push_back((uint32_t)(r + x));
        }
    }
}

// rho_I(J) of the planes (J <- result).  `marker_of(x, mask)` maps an image
// byte to the marker byte before clipping.
template <class MarkerOf>
void recon_from(Scratch &s, Plane out, Plane mask, int conn, MarkerOf marker_of) {
    Pad pd(mask);
    prepare(s, pd);
    for (int y = 0; y < pd.H; ++y) {
        const uint8_t *m = mask.row(y);
        const uint8_t *o = out.row(y);
        uint8_t *vr = &s.val[pd.at(y, 0)];
        uint8_t *mr = &s.msk[pd.at(y, 0)];
        for (int x = 0; x < pd.W; ++x) {
            mr[x] = m[x];
            vr[x] = std::min<uint8_t>(marker_of(o[x], m[x]), m[x]);
        }
    }
    seed_all(s, pd);
    flood(s, pd, conn);
}

int32_t find(std::vector<int32_t> &parent, int32_t a) {
    while (parent[a] != a) {
        parent[a] = parent[parent[a]];
        a = parent[a];
    }
    return a;
}

int32_t join(std::vector<int32_t> &parent, int32_t a, int32_t b) {
    a = find(parent, a);
    b = find(parent, b);
    if (a == b) return a;
    if (a < b) {
        parent[b] = a;
        return a;
    }
    parent[a] = b;
    return b;
}

// First raster pass: provisional labels into s.prov (H*W), equivalences in
// s.parent.  Returns the number of provisional labels.  After it, every
// parent[l] <= l.
int32_t provisional(Scratch &s, const Plane &img, int conn) {
    const int H = img.height, W = img.width;
    s.prov.assign((size_t)H * W, 0);
    s.parent.assign(1, 0);
    int32_t n = 0;
    for (int y = 0; y < H; ++y) {
        const uint8_t *r = img.row(y);
        int32_t *pr = &s.prov[(size_t)y * W];
        const int32_t *up = y > 0 ? &s.prov[(size_t)(y - 1) * W] : nullptr;
        for (int x = 0; x < W; ++x) {
            if (!r[x]) continue;
            const int32_t w = x > 0 ? pr[x - 1] : 0;
            const int32_t nb = up ? up[x] : 0;
            int32_t l;
            if (conn == 8) {
                const int32_t nw = (up && x > 0) ? up[x - 1] : 0;
                const int32_t ne = (up && x + 1 < W) ? up[x + 1] : 0;
                if (nb) {
                    l = nb;   // W, NW and NE all touch N under 8-connectivity
                } else if (ne) {
                    l = w ? join(s.parent, ne, w) : nw ? join(s.parent, ne, nw) : ne;
                } else {
                    l = w ? w : nw;
                }
            } else {
                l = (w && nb) ? join(s.parent, w, nb) : (w ? w : nb);
            }
            if (!l) {
                l = ++n;
                s.parent.push_back(l);
            }
            pr[x] = l;
        }
    }
    return n;
}

// Resolve every provisional label to the raster-order number of its
// component: parent[l] <= l, so one increasing pass reaches the roots; a root
// is the smallest label of its component, the label of its first pixel.
int32_t number_roots(Scratch &s, int32_t n) {
    int32_t count = 0;
    for (int32_t l = 1; l <= n; ++l) {
        const int32_t p = s.parent[l];
        s.parent[l] = (p == l) ? ++count : s.parent[p];
    }
    return count;
}

int32_t isqrt(int64_t d) {
    int64_t r = (int64_t)std::sqrt((double)d);
    while (r * r > d) --r;
    while ((r + 1) * (r + 1) <= d) ++r;
    return (int32_t)r;
}

int64_t floor_div(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

}  // namespace

void recon_dilate(Scratch *s, Plane marker, Plane mask, int conn) {
    recon_from(*s, marker, mask, conn, [](uint8_t j, uint8_t) { return j; });
    Pad pd(mask);
    for (int y = 0; y < pd.H; ++y) std::memcpy(marker.row(y), &s->val[pd.at(y, 0)], pd.W);
}

void hdome(Scratch *s, Plane img, int h, int conn) {
    recon_from(*s, img, img, conn, [h](uint8_t v, uint8_t) { return (uint8_t)(v > h ? v - h : 0); });
    Pad pd(img);
    for (int y = 0; y < pd.H; ++y) {
        uint8_t *r = img.row(y);
        const uint8_t *v = &s->val[pd.at(y, 0)];
        for (int x = 0; x < pd.W; ++x) r[x] = (uint8_t)(r[x] - v[x]);
    }
}

void regional_max(Scratch *s, Plane img, int conn) {
    recon_from(*s, img, img, conn, [](uint8_t v, uint8_t) { return (uint8_t)(v ? v - 1 : 0); });
    Pad pd(img);
    for (int y = 0; y < pd.H; ++y) {
        uint8_t *r = img.row(y);
        const uint8_t *v = &s->val[pd.at(y, 0)];
        for (int x = 0; x < pd.W; ++x) r[x] = r[x] != v[x] ? 255 : 0;
    }
}

void fill_holes(Scratch *s, Plane img, int conn) {
    Pad pd(img);
    prepare(*s, pd);
    const int H = pd.H, W = pd.W;
    for (int y = 0; y < H; ++y) {
        const uint8_t *r = img.row(y);
        uint8_t *mr = &s->msk[pd.at(y, 0)];
        uint8_t *vr = &s->val[pd.at(y, 0)];
        const bool edge_row = y == 0 || y == H - 1;
        for (int x = 0; x < W; ++x) {
            mr[x] = (uint8_t)(255 - r[x]);
            // the marker is the complemented image on the frame, 0 inside
            if (edge_row || x == 0 || x == W - 1) {
                vr[x] = mr[x];
                if (vr[x]) s->bucket[vr[x]].push_back((uint32_t)(pd.at(y, 0) + x));
            }
        }
    }
    flood(*s, pd, conn);
    for (int y = 0; y < H; ++y) {
        uint8_t *r = img.row(y);
        const uint8_t *v = &s->val[pd.at(y, 0)];
        for (int x = 0; x < W; ++x) r[x] = (uint8_t)(255 - v[x]);
    }
}

int32_t label(Scratch *s, Plane img, int32_t *labels, int64_t label_pitch, int conn) {
    const int32_t n = provisional(*s, img, conn);
    const int32_t count = number_roots(*s, n);
    for (int y = 0; y < img.height; ++y) {
        const int32_t *pr = &s->prov[(size_t)y * img.width];
        int32_t *o = labels + (int64_t)y * label_pitch;
        for (int x = 0; x < img.width; ++x) o[x] = pr[x] ? s->parent[pr[x]] : 0;
    }
    return count;
}

void area_threshold(Scratch *s, Plane img, int conn, int64_t lo, int64_t hi) {
    const int32_t n = provisional(*s, img, conn);
    const int32_t count = number_roots(*s, n);
    s->count.assign((size_t)count + 1, 0);
    const size_t N = (size_t)img.height * img.width;
    for (size_t i = 0; i < N; ++i)
        if (s->prov[i]) ++s->count[s->parent[s->prov[i]]];
    for (int y = 0; y < img.height; ++y) {
        uint8_t *r = img.row(y);
        const int32_t *pr = &s->prov[(size_t)y * img.width];
        for (int x = 0; x < img.width; ++x) {
            const int64_t a = pr[x] ? s->count[s->parent[pr[x]]] : -1;
            r[x] = (pr[x] && a >= lo && a <= hi) ? 255 : 0;
        }
    }
}

void distance2(Scratch *sc, Plane img, int32_t *dist2, int64_t dist_pitch) {
    const int H = img.height, W = img.width;
    const int32_t INF = H + W;   // above every finite column distance
    sc->g.assign((size_t)H * W, INF);
    int32_t *g = sc->g.data();
    bool any_zero = false;
    // column distances to the nearest 0 pixel above or below
    for (int y = 0; y < H; ++y) {
        const uint8_t *r = img.row(y);
        int32_t *gr = g + (size_t)y * W;
        const int32_t *ga = y > 0 ? g + (size_t)(y - 1) * W : nullptr;
        for (int x = 0; x < W; ++x) {
            if (!r[x]) {
                gr[x] = 0;
                any_zero = true;
            } else if (ga && ga[x] < INF) {
                gr[x] = ga[x] + 1;
            }
        }
    }
    if (!any_zero) {
        for (int y = 0; y < H; ++y)
            std::fill(dist2 + (int64_t)y * dist_pitch, dist2 + (int64_t)y * dist_pitch + W, 0x7fffffff);
        return;
    }
    for (int y = H - 2; y >= 0; --y) {
        int32_t *gr = g + (size_t)y * W;
        const int32_t *gb = g + (size_t)(y + 1) * W;
        for (int x = 0; x < W; ++x)
            if (gb[x] + 1 < gr[x]) gr[x] = gb[x] + 1;
    }
    // per row: lower envelope of the parabolas f_i(x) = (x - i)^2 + g(i)^2;
    // s[k] is the column of the k-th parabola of the envelope, t[k] the first x
    // where it is the lowest
    sc->s.resize(W);
    sc->t.resize(W);
    int32_t *sv = sc->s.data(), *tv = sc->t.data();
    for (int y = 0; y < H; ++y) {
        const int32_t *gr = g + (size_t)y * W;
        auto f = [gr](int64_t x, int64_t i) { return (x - i) * (x - i) + (int64_t)gr[i] * gr[i]; };
        // last x at which parabola i is not above parabola u (i < u)
        auto sep = [gr](int64_t i, int64_t u) {
            return floor_div(u * u - i * i + (int64_t)gr[u] * gr[u] - (int64_t)gr[i] * gr[i], 2 * (u - i));
        };
        int q = 0;
        sv[0] = 0;
        tv[0] = 0;
        for (int u = 1; u < W; ++u) {
            while (q >= 0 && f(tv[q], sv[q]) > f(tv[q], u)) --q;
            if (q < 0) {
                q = 0;
                sv[0] = u;
            } else {
                const int64_t w = 1 + sep(sv[q], u);
                if (w < W) {
                    ++q;
                    sv[q] = u;
                    tv[q] = (int32_t)w;
                }
            }
        }
        int32_t *o = dist2 + (int64_t)y * dist_pitch;
        for (int u = W - 1; u >= 0; --u) {
            const int64_t d = f(u, sv[q]);
            o[u] = (int32_t)std::min<int64_t>(d, 0x7fffffff);
            if (u == tv[q]) --q;
        }
    }
}

void pre_watershed(Scratch *s, Plane img, int conn) {
    const int H = img.height, W = img.width;
    s->d2.resize((size_t)H * W);
    distance2(s, img, s->d2.data(), W);
    for (int y = 0; y < H; ++y) {
        uint8_t *r = img.row(y);
        const int32_t *d = &s->d2[(size_t)y * W];
        for (int x = 0; x < W; ++x) r[x] = (uint8_t)std::min<int32_t>(isqrt(d[x]), 255);
    }
    regional_max(s, img, conn);
}

}  // namespace hostops

// Host-runtime check: drives the library's host code through its public C
// ABI on device 0 (frames with host and device buffers, a batch of uneven
// frames, the served form, the plane-set helpers, error paths) so that a
// build with host-side AddressSanitizer and UndefinedBehaviorSanitizer can
// watch every host path that a real run takes.  Exits non-zero on the first
// unexpected status; the sanitizers abort on the first report.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/fassmvs.h"

namespace {

int g_fail = 0;

#define CHECK(cond, what)                                                   \
    do {                                                                    \
        if (!(cond)) {                                                      \
            std::fprintf(stderr, "host check: %s failed (line %d)\n", what, __LINE__); \
            g_fail = 1;                                                     \
            return;                                                         \
        }                                                                   \
    } while (0)

// A textured image: sums of sines (deterministic), 8-bit.
std::vector<uint8_t> texture(int w, int h, double seed) {
    std::vector<uint8_t> img((size_t)w * h);
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            const double v = 128.0 + 50.0 * std::sin(0.31 * x + seed) * std::cos(0.23 * y - seed) +
                             30.0 * std::sin(0.071 * (x + 2 * y) + 3 * seed) + 20.0 * std::sin(0.9 * x * y * 1e-3);
            img[(size_t)y * w + x] = (uint8_t)std::lround(std::fmin(255.0, std::fmax(0.0, v)));
        }
    return img;
}

fassmvs_image image(const std::vector<uint8_t> &px, int w, int h, double tx) {
    fassmvs_image im;
    std::memset(&im, 0, sizeof(im));
    im.pixels = px.data();
    im.width = w;
    im.height = h;
    im.stride = w;
    im.R[0] = im.R[4] = im.R[8] = 1.0;
    im.t[0] = tx;
    return im;
}

fassmvs_plane_family fronto(int count) {
    fassmvs_plane_family f;
    std::memset(&f, 0, sizeof(f));
    f.n[2] = -1.0;
    f.delta_min = 20.0;
    f.delta_max = 200.0;
    f.count = count;
    return f;
}

struct Bundle {
    int w, h;
    std::vector<uint8_t> ref, v0, v1;
    fassmvs_image ims[3];
    int8_t side[2] = {-1, 1};
    double K[9];
    Bundle(int w_, int h_, double seed) : w(w_), h(h_), ref(texture(w_, h_, seed)), v0(texture(w_, h_, seed)),
                                          v1(texture(w_, h_, seed)) {
        ims[0] = image(ref, w, h, 0.0);
        ims[1] = image(v0, w, h, 0.5);
        ims[2] = image(v1, w, h, -0.5);
        const double K_[9] = {0.8 * w, 0, 0.5 * w, 0, 0.8 * w, 0.5 * h, 0, 0, 1};
        std::memcpy(K, K_, sizeof(K));
    }
};

void frames(fassmvs_handle *h) {
    Bundle b(256, 192, 0.3);
    fassmvs_plane_family fam = fronto(32);
    std::vector<float> d((size_t)b.w * b.h), n((size_t)b.w * b.h * 3), c((size_t)b.w * b.h);
    uint64_t t = 0;
    CHECK(fassmvs_submit_frame(h, &b.ims[0], &b.ims[1], b.side, 2, b.K, &fam, 1, FASSMVS_MEM_HOST, &t) == FASSMVS_OK,
          "host frame submit");
    CHECK(fassmvs_poll(h, t, d.data(), n.data(), c.data(), FASSMVS_MEM_HOST, -1) == FASSMVS_OK, "host frame poll");
    // device buffers in and out
    void *dimg[3] = {nullptr, nullptr, nullptr}, *dd = nullptr;
    for (int i = 0; i < 3; ++i) {
        CHECK(fassmvs_device_alloc(h, (size_t)b.w * b.h, &dimg[i]) == FASSMVS_OK, "device alloc");
        CHECK(fassmvs_memcpy(h, dimg[i], b.ims[i].pixels, (size_t)b.w * b.h, 0) == FASSMVS_OK, "upload");
    }
    CHECK(fassmvs_device_alloc(h, d.size() * 4, &dd) == FASSMVS_OK, "device alloc");
    fassmvs_image di[3];
    for (int i = 0; i < 3; ++i) {
        di[i] = b.ims[i];
        di[i].pixels = (const uint8_t *)dimg[i];
    }
    CHECK(fassmvs_submit_frame(h, &di[0], &di[1], b.side, 2, b.K, &fam, 1, FASSMVS_MEM_DEVICE, &t) == FASSMVS_OK,
          "device frame submit");
    CHECK(fassmvs_poll(h, t, (float *)dd, nullptr, nullptr, FASSMVS_MEM_DEVICE, -1) == FASSMVS_OK, "device poll");
    std::vector<float> d2(d.size());
    CHECK(fassmvs_memcpy(h, d2.data(), dd, d.size() * 4, 1) == FASSMVS_OK, "download");
    CHECK(std::memcmp(d.data(), d2.data(), d.size() * 4) == 0, "host and device frames agree");
    for (int i = 0; i < 3; ++i) fassmvs_device_free(h, dimg[i]);
    fassmvs_device_free(h, dd);
    // an explicit list and a depth range
    std::vector<double> list;
    for (int i = 0; i < 24; ++i) list.push_back(20.0 * std::pow(10.0, i / 23.0));
    fassmvs_plane_family fl = fronto(24);
    fl.delta = list.data();
    CHECK(fassmvs_submit_frame(h, &b.ims[0], &b.ims[1], b.side, 2, b.K, &fl, 1, FASSMVS_MEM_HOST, &t) == FASSMVS_OK,
          "list frame submit");
    CHECK(fassmvs_poll(h, t, d.data(), nullptr, nullptr, FASSMVS_MEM_HOST, -1) == FASSMVS_OK, "list frame poll");
    fassmvs_plane_family fr = fronto(16);
    fr.delta_min = fr.delta_max = 0.0;
    fr.depth_min = 25.0;
    fr.depth_max = 150.0;
    CHECK(fassmvs_submit_frame(h, &b.ims[0], &b.ims[1], b.side, 2, b.K, &fr, 1, FASSMVS_MEM_HOST, &t) == FASSMVS_OK,
          "range frame submit");
    CHECK(fassmvs_poll(h, t, d.data(), nullptr, nullptr, FASSMVS_MEM_HOST, -1) == FASSMVS_OK, "range frame poll");
    // errors: busy, unknown ticket, bad arguments
    CHECK(fassmvs_submit_frame(h, &b.ims[0], &b.ims[1], b.side, 2, b.K, &fam, 1, FASSMVS_MEM_HOST, &t) == FASSMVS_OK,
          "submit");
    uint64_t t2 = 0;
    CHECK(fassmvs_submit_frame(h, &b.ims[0], &b.ims[1], b.side, 2, b.K, &fam, 1, FASSMVS_MEM_HOST, &t2) ==
              FASSMVS_EBUSY,
          "busy");
    CHECK(fassmvs_poll(h, t + 9, nullptr, nullptr, nullptr, FASSMVS_MEM_HOST, 0) == FASSMVS_ENOTFOUND, "bad ticket");
    CHECK(fassmvs_poll(h, t, nullptr, nullptr, nullptr, FASSMVS_MEM_HOST, -1) == FASSMVS_OK, "poll");
    fassmvs_plane_family bad = fronto(1000);
    CHECK(fassmvs_submit_frame(h, &b.ims[0], &b.ims[1], b.side, 2, b.K, &bad, 1, FASSMVS_MEM_HOST, &t) ==
              FASSMVS_EINVAL,
          "plane cap");
    CHECK(std::strlen(fassmvs_last_error(h)) > 0, "error message");
}

void batch(fassmvs_handle *h) {
    Bundle a(256, 192, 0.1), b(320, 240, 0.7), c(200, 160, 1.3);
    fassmvs_plane_family f32 = fronto(32), f48 = fronto(48);
    fassmvs_frame fr[3];
    Bundle *bs[3] = {&a, &b, &c};
    for (int i = 0; i < 3; ++i) {
        std::memset(&fr[i], 0, sizeof(fr[i]));
        fr[i].ref = &bs[i]->ims[0];
        fr[i].views = &bs[i]->ims[1];
        fr[i].view_side = bs[i]->side;
        fr[i].n_views = 2;
        fr[i].K = bs[i]->K;
        fr[i].families = i == 1 ? &f48 : &f32;
        fr[i].n_families = 1;
        fr[i].n_levels = i == 2 ? 1 : 2;
        fr[i].window_labels = -1;
    }
    for (int rep = 0; rep < 2; ++rep) {
        uint64_t t = 0;
        CHECK(fassmvs_submit_batch(h, fr, 3, FASSMVS_MEM_HOST, &t) == FASSMVS_OK, "batch submit");
        for (int i = 0; i < 3; ++i) {
            std::vector<float> d((size_t)bs[i]->w * bs[i]->h);
            CHECK(fassmvs_poll_batch(h, t, i, d.data(), nullptr, nullptr, FASSMVS_MEM_HOST, -1) == FASSMVS_OK,
                  "batch poll");
        }
    }
    int32_t rpt = 0, blocks = 0, groups = 0, graph = 0;
    double ms = 0;
    CHECK(fassmvs_batch_tuning(h, &rpt, &blocks, &groups, &graph, &ms) == FASSMVS_OK, "batch tuning");
    CHECK(rpt == 0 || rpt == 4 || rpt == 8, "tuned rows");
}

void served() {
    fassmvs_config cfg;
    fassmvs_config_default(&cfg);
    cfg.n_levels = 2;
    fassmvs_server *s = nullptr;
    if (fassmvs_server_create(&cfg, 2, 0, &s) != FASSMVS_OK) {
        std::fprintf(stderr, "host check: server create failed\n");
        g_fail = 1;
        return;
    }
    Bundle a(256, 192, 0.2), b(192, 128, 0.9);
    fassmvs_plane_family f = fronto(32);
    int32_t sa = 0, sb = 0;
    CHECK(fassmvs_server_open_stream(s, a.K, a.w, a.h, &f, 1, 3, 0.4, &sa) == FASSMVS_OK, "open stream");
    CHECK(fassmvs_server_open_stream(s, b.K, b.w, b.h, &f, 1, 3, 0.4, &sb) == FASSMVS_OK, "open stream");
    int submitted = 0;
    for (int i = 0; i < 6; ++i) {
        const double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        const double t[3] = {0.5 * i, 0, 0};
        uint64_t id = 0;
        std::vector<uint8_t> ia = texture(a.w, a.h, 0.2 + 0.01 * i), ib = texture(b.w, b.h, 0.9 + 0.01 * i);
        CHECK(fassmvs_server_submit(s, sa, ia.data(), a.w, R, t, &id) == FASSMVS_OK, "served submit");
        CHECK(fassmvs_server_submit(s, sb, ib.data(), b.w, R, t, &id) == FASSMVS_OK, "served submit");
        submitted += 2;
    }
    int with_maps = 0;
    for (int i = 0; i < submitted; ++i) {
        fassmvs_server_result r;
        CHECK(fassmvs_server_next(s, -1, &r) == FASSMVS_OK, "served next");
        if (r.status == FASSMVS_OK) {
            std::vector<float> d((size_t)r.width * r.height);
            CHECK(fassmvs_server_fetch(s, r.request_id, d.data(), nullptr, nullptr, FASSMVS_MEM_HOST) == FASSMVS_OK,
                  "served fetch");
            ++with_maps;
        }
    }
    CHECK(with_maps >= submitted - 2, "served maps");
    CHECK(fassmvs_server_close_stream(s, sa) == FASSMVS_OK, "close stream");
    CHECK(fassmvs_server_close_stream(s, sb) == FASSMVS_OK, "close stream");
    fassmvs_server_destroy(s);
}

void planes() {
    const double K[9] = {400, 0, 160, 0, 400, 120, 0, 0, 1};
    const double n[3] = {0, 0, -1};
    double out[2] = {0, 0};
    CHECK(fassmvs_bounding_planes(K, 320, 240, n, 10.0, 100.0, out) == FASSMVS_OK, "bounding planes");
    CHECK(std::fabs(out[0] - 10.0) < 1e-9 && std::fabs(out[1] - 100.0) < 1e-9, "fronto bounding planes");
    CHECK(fassmvs_bounding_planes(K, 320, 240, n, 100.0, 10.0, out) == FASSMVS_EINVAL, "bad range");
    const double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    const double t[3] = {-1.0, 0, 0};
    std::vector<double> d(4096);
    int32_t count = 0;
    CHECK(fassmvs_cross_ratio_planes(K, 320, 240, R, t, n, 10.0, 100.0, 4096, d.data(), &count) == FASSMVS_OK,
          "cross-ratio planes");
    CHECK(count > 2, "cross-ratio count");
    CHECK(fassmvs_cross_ratio_planes(K, 320, 240, R, t, n, 10.0, 100.0, 2, d.data(), &count) ==
              FASSMVS_EUNSUPPORTED,
          "cross-ratio capacity");
    fassmvs_config cfg;
    fassmvs_config_default(&cfg);
    fassmvs_plane_family f = fronto(64);
    uint64_t bytes = 0;
    CHECK(fassmvs_frame_footprint(&cfg, 640, 480, 4, &f, 1, &bytes) == FASSMVS_OK && bytes > 0, "footprint");
}

}  // namespace

int main() {
    fassmvs_config cfg;
    fassmvs_config_default(&cfg);
    cfg.n_levels = 2;
    cfg.window_labels = 16;
    cfg.profile = 1;
    fassmvs_handle *h = nullptr;
    if (fassmvs_create(&cfg, &h) != FASSMVS_OK) {
        std::fprintf(stderr, "host check: create failed: %s\n", fassmvs_last_error(nullptr));
        return 1;
    }
    frames(h);
    if (!g_fail) batch(h);
    fassmvs_destroy(h);
    if (!g_fail) served();
    if (!g_fail) planes();
    std::printf(g_fail ? "host check: FAILED\n" : "host check: ok\n");
    std::fflush(stdout);
    return g_fail;
}

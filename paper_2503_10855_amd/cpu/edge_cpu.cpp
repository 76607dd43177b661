// edge_cpu.cpp -- a tuned multi-core fp32 CPU implementation of the EDGE
// pipeline, the comparison point for the GPU path on the host's cores (the
// paper's multicore! pattern, Use and Impact of Schedules: the work is
// chunked into units that run as parallel tasks, each a sequential,
// vectorisable loop nest).
//
// A unit is a band of up to 128 rows of one image.  Phase 1 computes, for
// every pixel of the band, the stages the band needs (horizontal then
// vertical blur, Laplacian sign, Sobel G^2, zero crossing, each reading its
// input at clamped coordinates) into row planes of thread-local scratch,
// stores code = G^2 where Z else -1, and the band's max G^2.  Phase 2 turns
// codes into the mask against theta * sqrt(max).  Units are taken from an
// atomic counter by std::threads.  Row loops run over contiguous floats so
// the compiler vectorises them.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

namespace {

constexpr int kBand = 128;

struct Image {
    const float* src;
    int64_t H, W, pitch;
    uint8_t* mask;
    int64_t mpitch;
};

inline int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

struct Scratch {
    std::vector<float> hb, b, g2;  // planes of rows
    std::vector<uint8_t> s;              // sign of L
    std::vector<float> row;              // one padded input row
};

// Phase 1 on rows [y0, y1) of one image.  Returns the band's max G^2.
float band_codes(const Image& im, int64_t y0, int64_t y1, const float* g, int ks,
                 float* code, Scratch& sc) {
    const int r = ks / 2;
    const int64_t H = im.H, W = im.W;
    // Rows each stage needs: Z of [y0, y1) needs L (and S) of [y0-1, y1+1);
    // L and G^2 need B of [y0-2, y1+2); B needs the horizontal blur of
    // [y0-2-r, y1+2+r).  Rows outside the image are the clamped rows of
    // the stage's own input, as in the oracle.
    const int64_t bl0 = y0 - 2, bl1 = y1 + 2;   // B rows (unclamped ids)
    const int64_t nb = bl1 - bl0;
    const int64_t Wp = W + 2;                    // B rows padded by one column
    sc.b.resize((size_t)(nb * Wp));
    sc.hb.resize((size_t)(ks * W));
    sc.row.resize((size_t)(W + 2 * r));
    std::vector<int64_t> hb_row(ks, INT64_MIN);  // which input row each hb slot holds
    auto hblur = [&](int64_t iy, float* out) {
        const float* in = im.src + clampi(iy, 0, H - 1) * im.pitch;
        float* pr = sc.row.data();
        for (int k = 0; k < r; ++k) {
            pr[k] = in[0];
            pr[W + r + k] = in[W - 1];
        }
        std::memcpy(pr + r, in, sizeof(float) * W);
        for (int64_t x = 0; x < W; ++x) out[x] = g[0] * pr[x];
        for (int k = 1; k < ks; ++k) {
            const float gk = g[k];
            const float* pk = pr + k;
            for (int64_t x = 0; x < W; ++x) out[x] += gk * pk[x];
        }
    };
    // B rows: B(y) for y in [bl0, bl1), each B row computed for the clamped
    // row id (so rows above / below the image repeat row 0 / H-1).
    for (int64_t i = 0; i < nb; ++i) {
        const int64_t yb = clampi(bl0 + i, 0, H - 1);
        float* out = sc.b.data() + i * Wp + 1;
        for (int64_t x = 0; x < W; ++x) out[x] = 0.0f;
        for (int k = 0; k < ks; ++k) {
            const int64_t iy = yb + k - r;
            const int slot = (int)(((clampi(iy, 0, H - 1)) % ks + ks) % ks);
            float* h = sc.hb.data() + (int64_t)slot * W;
            if (hb_row[slot] != clampi(iy, 0, H - 1)) {
                hblur(iy, h);
                hb_row[slot] = clampi(iy, 0, H - 1);
            }
            const float gk = g[k];
            for (int64_t x = 0; x < W; ++x) out[x] += gk * h[x];
        }
        out[-1] = out[0];
        out[W] = out[W - 1];
    }
    // L sign and G^2 for rows [y0-1, y1+1) (clamped ids for L).
    const int64_t nl = (y1 + 1) - (y0 - 1);
    const int64_t Sp = W + 2;
    sc.s.resize((size_t)(nl * Sp));
    sc.g2.resize((size_t)((y1 - y0) * W));
    for (int64_t i = 0; i < nl; ++i) {
        const int64_t yl = clampi(y0 - 1 + i, 0, H - 1);
        // B rows yl-1, yl, yl+1 (clamped) sit at index (clamped row - bl0).
        const float* bn = sc.b.data() + (clampi(yl - 1, 0, H - 1) - bl0) * Wp + 1;
        const float* bc = sc.b.data() + (yl - bl0) * Wp + 1;
        const float* bs = sc.b.data() + (clampi(yl + 1, 0, H - 1) - bl0) * Wp + 1;
        uint8_t* s = sc.s.data() + i * Sp + 1;
        for (int64_t x = 0; x < W; ++x) {
            const float l = ((bn[x] + bs[x]) + (bc[x - 1] + bc[x + 1])) - 4.0f * bc[x];
            s[x] = l > 0.0f;
        }
        s[-1] = s[0];
        s[W] = s[W - 1];
        const int64_t yg = y0 - 1 + i;
        if (yg >= y0 && yg < y1) {
            float* g2 = sc.g2.data() + (yg - y0) * W;
            for (int64_t x = 0; x < W; ++x) {
                const float gx = (bn[x + 1] - bn[x - 1]) + 2.0f * (bc[x + 1] - bc[x - 1]) +
                                 (bs[x + 1] - bs[x - 1]);
                const float gy = (bs[x - 1] + 2.0f * bs[x] + bs[x + 1]) -
                                 (bn[x - 1] + 2.0f * bn[x] + bn[x + 1]);
                g2[x] = gx * gx + gy * gy;
            }
        }
    }
    // Z and the code for [y0, y1).
    float mx = 0.0f;
    for (int64_t y = y0; y < y1; ++y) {
        const int64_t i = y - (y0 - 1);
        const uint8_t* sn = sc.s.data() + (clampi(y - 1, 0, H - 1) - (y0 - 1)) * Sp + 1;
        const uint8_t* sm = sc.s.data() + i * Sp + 1;
        const uint8_t* ss = sc.s.data() + (clampi(y + 1, 0, H - 1) - (y0 - 1)) * Sp + 1;
        const float* g2 = sc.g2.data() + (y - y0) * W;
        float* c = code + y * W;
        for (int64_t x = 0; x < W; ++x) {
            const int any = sn[x - 1] | sn[x] | sn[x + 1] | sm[x - 1] | sm[x] | sm[x + 1] |
                            ss[x - 1] | ss[x] | ss[x + 1];
            const int all = sn[x - 1] & sn[x] & sn[x + 1] & sm[x - 1] & sm[x] & sm[x + 1] &
                            ss[x - 1] & ss[x] & ss[x + 1];
            const float v = g2[x];
            mx = v > mx ? v : mx;
            c[x] = (any & !all) ? v : -1.0f;
        }
    }
    return mx;
}

}  // namespace

extern "C" {

// Masks of n images (host memory; src row pitch and mask row pitch in
// elements), computed with `threads` worker threads.  d_max (nullable)
// receives M = max G per image.  Returns 0, or -1 on bad arguments.
int hx_cpu_edge_detect_many(int n, const float* const* src, const int64_t* H,
                            const int64_t* W, const int64_t* pitch, uint8_t* const* mask,
                            const int64_t* mpitch, int ksize, double sigma, double theta,
                            int threads, double* d_max) {
    if (n < 0 || ksize < 1 || ksize > 15 || !(ksize & 1) || sigma <= 0.0 || threads < 1)
        return -1;
    std::vector<Image> ims(n);
    for (int i = 0; i < n; ++i) {
        if (!src[i] || !mask[i] || H[i] < 1 || W[i] < 1 || pitch[i] < W[i] || mpitch[i] < W[i])
            return -1;
        ims[i] = Image{src[i], H[i], W[i], pitch[i], mask[i], mpitch[i]};
    }
    // Gaussian taps: sampled, normalised in double, used in fp32.
    float g[15];
    {
        const int r = ksize / 2;
        double w[15], sum = 0.0;
        for (int k = 0; k < ksize; ++k) {
            const double d = k - r;
            w[k] = std::exp(-(d * d) / (2.0 * sigma * sigma));
            sum += w[k];
        }
        for (int k = 0; k < ksize; ++k) g[k] = (float)(w[k] / sum);
    }
    struct Unit { int img; int64_t y0, y1; };
    std::vector<Unit> units;
    std::vector<size_t> code_off(n);
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        code_off[i] = total;
        total += (size_t)(ims[i].H * ims[i].W);
        for (int64_t y = 0; y < ims[i].H; y += kBand)
            units.push_back(Unit{i, y, std::min<int64_t>(ims[i].H, y + kBand)});
    }
    // Every code is written in phase 1: no need to clear the plane first.
    std::unique_ptr<float[]> code(new float[total]);
    std::vector<float> umax(units.size(), 0.0f);
    std::vector<float> thr2(n, 0.0f);
    // Runs body(unit, worker index) over every unit on `threads` workers.
    auto run = [&](auto&& body) {
        std::atomic<size_t> next{0};
        auto worker = [&](int t) {
            for (size_t u; (u = next.fetch_add(1)) < units.size();) body(u, t);
        };
        std::vector<std::thread> pool;
        for (int t = 1; t < threads; ++t) {
            try {
                pool.emplace_back(worker, t);
            } catch (...) {  // fewer threads: the others take the units
                break;
            }
        }
        worker(0);
        for (auto& t : pool) t.join();
    };
    std::vector<Scratch> scr(threads);
    run([&](size_t u, int t) {
        const Unit& un = units[u];
        umax[u] = band_codes(ims[un.img], un.y0, un.y1, g, ksize, code.get() + code_off[un.img],
                             scr[t]);
    });
    std::vector<float> m2(n, 0.0f);
    for (size_t u = 0; u < units.size(); ++u)
        m2[units[u].img] = std::max(m2[units[u].img], umax[u]);
    for (int i = 0; i < n; ++i) {
        const float tau = (float)theta * std::sqrt(m2[i]);
        thr2[i] = tau * tau;
        if (d_max) d_max[i] = std::sqrt((double)m2[i]);
    }
    run([&](size_t u, int) {
        const Unit& un = units[u];
        const Image& im = ims[un.img];
        const float t = thr2[un.img];
        for (int64_t y = un.y0; y < un.y1; ++y) {
            const float* c = code.get() + code_off[un.img] + y * im.W;
            uint8_t* m = im.mask + y * im.mpitch;
            for (int64_t x = 0; x < im.W; ++x) m[x] = c[x] > t;
        }
    });
    return 0;
}

}  // extern "C"

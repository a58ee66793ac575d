// Host-side set-up of an as-S_N problem (FP64).  See asn_host.hpp.
#include "asn_host.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>

namespace asn {

// Legendre P_n(x) and P_n'(x) by the three-term recurrence.
static void legendre(int n, double x, double& p, double& dp) {
    double p0 = 1.0, p1 = x;
    for (int j = 2; j <= n; ++j) {
        double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
    }
    p = (n == 0) ? 1.0 : p1;
    dp = (n == 0) ? 0.0 : n * (x * p1 - p0) / (x * x - 1.0);
}

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    if (n == 1) {
        w[0] = 2.0;
        return;
    }
    // Newton's method on P_n from the Chebyshev-like guesses cos(pi (i + 3/4) / (n + 1/2)),
    // exploiting the symmetry x_{n-1-i} = -x_i.
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double p = 0.0, dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            legendre(n, z, p, dp);
            double dz = p / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        legendre(n, z, p, dp);
        double wi = 2.0 / ((1.0 - z * z) * dp * dp);
        x[n - 1 - i] = z;
        x[i] = -z;
        w[n - 1 - i] = wi;
        w[i] = wi;
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
}

void product_quadrature(int n_polar, int n_azim, std::vector<double>& omega,
                        std::vector<double>& w) {
    std::vector<double> mu, g;
    gauss_legendre(n_polar, mu, g);
    const int Q = n_polar * n_azim;
    omega.assign(3 * (size_t)Q, 0.0);
    w.assign(Q, 0.0);
    const double dphi = 2.0 * M_PI / n_azim;
    for (int i = 0; i < n_polar; ++i) {
        const double s = std::sqrt(1.0 - mu[i] * mu[i]);
        for (int k = 0; k < n_azim; ++k) {
            const int q = i * n_azim + k;
            const double phi = (k + 0.5) * dphi;
            omega[3 * q + 0] = s * std::cos(phi);
            omega[3 * q + 1] = s * std::sin(phi);
            omega[3 * q + 2] = mu[i];
            w[q] = g[i] * dphi;
        }
    }
}

namespace {

struct V3 {
    double x, y, z;
};
V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
V3 unit(V3 a) { return (1.0 / std::sqrt(dot(a, a))) * a; }

// Solid angle of the spherical triangle a, b, c (unit vectors).
double solid_angle(V3 a, V3 b, V3 c) {
    const double num = std::fabs(dot(a, cross(b, c)));
    const double den = 1.0 + dot(a, b) + dot(b, c) + dot(c, a);
    return 2.0 * std::atan2(num, den);
}

}  // namespace

void icosahedron_quadrature(int order, std::vector<double>& omega, std::vector<double>& w) {
    const int m = order - 1;
    // 12 vertices: north pole, ring at z = 1/sqrt5 (azimuth 72 k deg), ring at
    // z = -1/sqrt5 (azimuth 72 k + 36 deg), south pole.
    std::array<V3, 12> vx;
    const double zr = 1.0 / std::sqrt(5.0), rr = 2.0 / std::sqrt(5.0);
    vx[0] = {0.0, 0.0, 1.0};
    vx[11] = {0.0, 0.0, -1.0};
    for (int k = 0; k < 5; ++k) {
        const double a = 2.0 * M_PI * k / 5.0, b = a + M_PI / 5.0;
        vx[1 + k] = {rr * std::cos(a), rr * std::sin(a), zr};
        vx[6 + k] = {rr * std::cos(b), rr * std::sin(b), -zr};
    }
    std::vector<std::array<int, 3>> faces;
    for (int k = 0; k < 5; ++k) {
        const int u0 = 1 + k, u1 = 1 + (k + 1) % 5, l0 = 6 + k, l1 = 6 + (k + 1) % 5;
        faces.push_back({0, u0, u1});
        faces.push_back({u0, l0, u1});
        faces.push_back({u1, l0, l1});
        faces.push_back({11, l1, l0});
    }
    // Nodes shared by neighbouring faces are merged by their rounded coordinates.
    std::map<std::array<long long, 3>, int> index;
    std::vector<V3> nodes;
    auto node_of = [&](V3 p) {
        p = unit(p);
        const std::array<long long, 3> key = {std::llround(p.x * 1e11), std::llround(p.y * 1e11),
                                              std::llround(p.z * 1e11)};
        auto it = index.find(key);
        if (it != index.end()) return it->second;
        const int id = (int)nodes.size();
        index.emplace(key, id);
        nodes.push_back(p);
        return id;
    };
    std::vector<std::array<int, 3>> tris;
    for (const auto& f : faces) {
        const V3 A = vx[f[0]], B = vx[f[1]], C = vx[f[2]];
        std::vector<int> grid((size_t)(m + 1) * (m + 1), -1);
        auto at = [&](int i, int j) -> int& { return grid[(size_t)i * (m + 1) + j]; };
        for (int i = 0; i <= m; ++i)
            for (int j = 0; i + j <= m; ++j)
                at(i, j) = node_of(A + ((double)i / m) * (B - A) + ((double)j / m) * (C - A));
        for (int i = 0; i < m; ++i)
            for (int j = 0; i + j < m; ++j) {
                tris.push_back({at(i, j), at(i + 1, j), at(i, j + 1)});
                if (i + j + 2 <= m) tris.push_back({at(i + 1, j), at(i + 1, j + 1), at(i, j + 1)});
            }
    }
    const size_t N = nodes.size();
    // Centres of the triangles around every node, walked in angular order.
    std::vector<std::vector<V3>> fan(N);
    for (const auto& t : tris) {
        const V3 g = unit(nodes[t[0]] + nodes[t[1]] + nodes[t[2]]);
        for (int v : t) fan[v].push_back(g);
    }
    std::vector<double> area(N, 0.0);
    for (size_t v = 0; v < N; ++v) {
        const V3 p = nodes[v];
        const V3 ref = std::fabs(p.z) < 0.9 ? V3{0.0, 0.0, 1.0} : V3{1.0, 0.0, 0.0};
        const V3 e1 = unit(cross(p, ref)), e2 = cross(p, e1);
        std::vector<std::pair<double, V3>> ring;
        for (const V3& g : fan[v]) ring.push_back({std::atan2(dot(g, e2), dot(g, e1)), g});
        std::sort(ring.begin(), ring.end(),
                  [](const std::pair<double, V3>& a, const std::pair<double, V3>& b) {
                      return a.first < b.first;
                  });
        double s = 0.0;
        for (size_t i = 0; i < ring.size(); ++i)
            s += solid_angle(p, ring[i].second, ring[(i + 1) % ring.size()].second);
        area[v] = s;
    }
    // Order: decreasing z, then increasing azimuth (both compared after rounding).
    std::vector<size_t> perm(N);
    for (size_t i = 0; i < N; ++i) perm[i] = i;
    auto zkey = [&](size_t i) { return std::llround(nodes[i].z * 1e9); };
    auto akey = [&](size_t i) {
        double a = std::atan2(nodes[i].y, nodes[i].x);
        if (a < 0) a += 2.0 * M_PI;
        return std::llround(a * 1e9);
    };
    std::sort(perm.begin(), perm.end(), [&](size_t a, size_t b) {
        if (zkey(a) != zkey(b)) return zkey(a) > zkey(b);
        return akey(a) < akey(b);
    });
    omega.assign(3 * N, 0.0);
    w.assign(N, 0.0);
    for (size_t i = 0; i < N; ++i) {
        const V3 p = nodes[perm[i]];
        omega[3 * i] = p.x;
        omega[3 * i + 1] = p.y;
        omega[3 * i + 2] = p.z;
        w[i] = area[perm[i]];
    }
}

bool kernel_matrix(int Q, const double* om, const double* w, double eps, int mode,
                   std::vector<double>& K, std::string& err) {
    K.assign((size_t)Q * Q, 0.0);
    for (int q = 0; q < Q; ++q) {
        for (int p = 0; p < Q; ++p) {
            const double c = om[3 * q] * om[3 * p] + om[3 * q + 1] * om[3 * p + 1] +
                             om[3 * q + 2] * om[3 * p + 2];
            const double y = (1.0 - c) / eps;
            K[(size_t)q * Q + p] = std::exp(-y * y);
        }
    }
    if (mode == 1) {  // c_q^(eps) = 1 / sum_p w_p s_qp
        for (int q = 0; q < Q; ++q) {
            double* row = &K[(size_t)q * Q];
            double s = 0.0;
            for (int p = 0; p < Q; ++p) s += w[p] * row[p];
            for (int p = 0; p < Q; ++p) row[p] = w[p] * row[p] / s;
        }
        return true;
    }
    // Symmetric scaling: find d > 0 with d_q sum_p S_qp w_p d_p = 1 for all q.
    std::vector<double> d(Q), rows(Q);
    for (int q = 0; q < Q; ++q) {
        double s = 0.0;
        for (int p = 0; p < Q; ++p) s += K[(size_t)q * Q + p] * w[p];
        d[q] = 1.0 / std::sqrt(s);
    }
    bool ok = false;
    for (int it = 0; it < 10000; ++it) {
        double worst = 0.0;
        for (int q = 0; q < Q; ++q) {
            double s = 0.0;
            const double* row = &K[(size_t)q * Q];
            for (int p = 0; p < Q; ++p) s += row[p] * w[p] * d[p];
            rows[q] = d[q] * s;
            worst = std::fmax(worst, std::fabs(rows[q] - 1.0));
        }
        if (worst <= 1e-14) {
            ok = true;
            break;
        }
        for (int q = 0; q < Q; ++q) d[q] /= std::sqrt(rows[q]);
    }
    if (!ok) {
        err = "symmetric kernel scaling did not converge";
        return false;
    }
    for (int q = 0; q < Q; ++q)
        for (int p = 0; p < Q; ++p) K[(size_t)q * Q + p] *= d[q] * w[p] * d[p];
    return true;
}

void cfl_time_step(int Q, const double* om, double dx, double dy, double cfl, double t_final,
                   double& dt, int64_t& n) {
    double rate = 0.0;
    for (int q = 0; q < Q; ++q)
        rate = std::fmax(rate, std::fabs(om[3 * q]) / dx + std::fabs(om[3 * q + 1]) / dy);
    const double dt_max = cfl / rate;
    n = (int64_t)std::ceil(t_final / dt_max * (1.0 - 1e-12));
    if (n < 1) n = 1;
    dt = t_final / (double)n;
}

double stability_rate(int Q, const double* om, const double* K, double dx, double dy, int64_t C,
                      const float* sigma_a, const float* sigma_s, const float* sigma_as) {
    double r = 0.0, kmin = 1.0;
    for (int q = 0; q < Q; ++q) {
        r = std::fmax(r, std::fabs(om[3 * q]) / dx + std::fabs(om[3 * q + 1]) / dy);
        kmin = std::fmin(kmin, K[(size_t)q * Q + q]);
    }
    const double g = 2.0 * (1.0 - kmin);
    double m = 0.0;
    for (int64_t c = 0; c < C; ++c)
        m = std::fmax(m, (double)sigma_a[c] + (double)sigma_s[c] + g * (double)sigma_as[c]);
    return 2.0 * r + m;
}

void stiff_time_step(int Q, const double* om, double dx, double dy, double srate, double cfl,
                     double t_final, double& dt, int64_t& n) {
    double rate = 0.0;
    for (int q = 0; q < Q; ++q)
        rate = std::fmax(rate, std::fabs(om[3 * q]) / dx + std::fabs(om[3 * q + 1]) / dy);
    const double dt_max = std::fmin(cfl / rate, 2.0 * cfl / srate);
    n = (int64_t)std::ceil(t_final / dt_max * (1.0 - 1e-12));
    if (n < 1) n = 1;
    dt = t_final / (double)n;
}

static uint32_t f2u(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}
static float u2f(uint32_t u) {
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

uint16_t float_to_bf16_rne(float f) {
    uint32_t u = f2u(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Shift right by s bits rounding to nearest, ties to even.
static uint32_t shift_rne(uint32_t m, int s) {
    if (s <= 0) return m;
    if (s > 31) return 0;
    const uint32_t q = m >> s;
    const uint32_t rem = m & ((1u << s) - 1u);
    const uint32_t half = 1u << (s - 1);
    return (rem > half || (rem == half && (q & 1u))) ? q + 1u : q;
}

uint16_t float_to_half_rne(float f) {
    const uint32_t u = f2u(f);
    const uint16_t sign = (uint16_t)((u >> 16) & 0x8000u);
    const uint32_t a = u & 0x7FFFFFFFu;
    if (a >= 0x7F800000u) return sign | 0x7C00u | (a > 0x7F800000u ? 0x200u : 0u);
    if (a < 0x00800000u) return sign;  // float subnormals are far below the half range
    const int e = (int)(a >> 23) - 127 + 15;  // biased half exponent
    const uint32_t m = (a & 0x7FFFFFu) | 0x800000u;
    if (e >= 1) {
        uint32_t r = shift_rne(m, 13);  // 24 -> 11 significant bits
        int ee = e;
        if (r == 0x800u) {
            r >>= 1;
            ++ee;
        }
        if (ee >= 31) return sign | 0x7C00u;
        return sign | (uint16_t)(ee << 10) | (uint16_t)(r & 0x3FFu);
    }
    const uint32_t r = shift_rne(m, 13 + 1 - e);  // subnormal half (may round up to 0x400)
    return sign | (uint16_t)r;
}

float bf16_to_float(uint16_t h) { return u2f((uint32_t)h << 16); }

float half_to_float(uint16_t h) {
    const uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
    const uint32_t e = (h >> 10) & 0x1Fu;
    const uint32_t m = h & 0x3FFu;
    if (e == 0) return (sign ? -1.0f : 1.0f) * std::ldexp((float)m, -24);
    if (e == 31) return u2f(sign | 0x7F800000u | (m << 13));
    return u2f(sign | ((e - 15 + 127) << 23) | (m << 13));
}

}  // namespace asn

namespace asn {

bool band_form(int levels, int azim, const float* K32, int max_reach, int narrow_max,
               BandForm& out) {
    if (levels < 1 || azim < 2 || azim % 2 || azim > 126 || max_reach > 3) return false;
    const int Q = levels * azim;
    auto wrap = [azim](int d) { return ((d % azim) + azim) % azim; };
    // every row equals the first row of its level, shifted by the row's azimuth
    for (int i = 0; i < levels; ++i)
        for (int k = 1; k < azim; ++k) {
            const float* r0 = K32 + (size_t)(i * azim) * Q;
            const float* rk = K32 + (size_t)(i * azim + k) * Q;
            for (int j = 0; j < levels; ++j)
                for (int kp = 0; kp < azim; ++kp)
                    if (rk[j * azim + kp] != r0[j * azim + wrap(kp - k)]) return false;
        }
    int reach = 0;
    for (int i = 0; i < levels; ++i)
        for (int j = 0; j < levels; ++j)
            for (int kp = 0; kp < azim; ++kp)
                if (K32[(size_t)(i * azim) * Q + j * azim + kp] != 0.f)
                    reach = std::max(reach, std::abs(i - j));
    if (reach > max_reach) return false;
    out.levels = levels;
    out.azim = azim;
    out.reach = reach;
    out.cmax = 0;
    out.desc.assign((size_t)levels * 8, 0u);
    out.range.assign((size_t)levels * 2, 0);
    out.coef.clear();
    for (int i = 0; i < levels; ++i) {
        const int base = (int)out.coef.size();
        int n = 0;
        for (int k = 0; k < 2 * reach + 1; ++k) {
            const int j = i + k - reach;
            if (j < 0 || j >= levels) continue;
            const float* r0 = K32 + (size_t)(i * azim) * Q + j * azim;
            int s = -1;
            for (int kp = 0; kp < azim; ++kp)
                if (r0[kp] != 0.f) s = std::max(s, std::min(kp, azim - kp));
            if (s < 0) continue;
            const bool ring = 2 * s + 1 >= azim;
            const int start4 = ((int)out.coef.size() - base) / 4;
            if (start4 > 127) return false;
            const uint32_t c = (uint32_t)(ring ? azim / 2 : s) | (ring || s > narrow_max ? 64u : 0u) |
                               (ring ? 128u : 0u) | ((uint32_t)k << 8) | ((uint32_t)start4 << 11);
            out.desc[(size_t)i * 8 + 1 + n] = c;
            ++n;
            int lo = 0, len = 0;
            band_run(c, azim, lo, len);
            for (int t = 0; t < len; ++t) out.coef.push_back(r0[wrap(lo + t)]);
            while (out.coef.size() % 4) out.coef.push_back(0.f);
        }
        out.desc[(size_t)i * 8] = (uint32_t)n;
        out.range[2 * (size_t)i] = base;
        out.range[2 * (size_t)i + 1] = (int)out.coef.size() - base;
        if ((int)out.coef.size() - base > 508) return false;
        out.cmax = std::max(out.cmax, (int)out.coef.size() - base);
    }
    return true;
}

void band_lp_fragments(const BandForm& bf, int level, int pair, int dtype,
                       std::vector<uint16_t>& out) {
    const int azim = bf.azim;
    const uint32_t code = bf.desc[(size_t)level * 8 + 1 + pair];
    int lo = 0, len = 0;
    band_run(code, azim, lo, len);
    const int start = 4 * (int)((code >> 11) & 127u) + bf.range[2 * (size_t)level];
    std::vector<float> c((size_t)azim, 0.f);   // c(delta), delta = 0 .. azim - 1
    for (int t = 0; t < len; ++t) c[(size_t)(((lo + t) % azim + azim) % azim)] = bf.coef[(size_t)start + t];
    for (int f = 0; f < azim / 16; ++f)
        for (int l = 0; l < 64; ++l)
            for (int t = 0; t < 8; ++t) {
                const int m = l % 16, k = 8 * (l / 16) + t;
                const float v = c[(size_t)(((16 * f + k - m) % azim + azim) % azim)];
                out.push_back(dtype == 1 ? float_to_bf16_rne(v) : float_to_half_rne(v));
            }
}

}  // namespace asn

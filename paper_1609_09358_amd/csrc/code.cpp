// code.cpp -- construction of polar codes (frozen set, CRC tables) and the
// non-kernel parts of the C ABI: errors, code handles, parameter queries.
//
// Frozen-set construction: the paper decodes an arbitrary given frozen vector
// (Sec. II).  When none is given, the Gaussian approximation of density
// evolution is used (Chung, Richardson, Urbanke 2001; Trifonov 2012): the
// channel LLR mean 2/sigma^2 is pushed through n polarisation steps, the
// check-node side mapping m to phi^{-1}(1 - (1 - phi(m))^2) and the
// variable-node side to 2m; the first step decides the most significant index
// bit.  phi uses the two-piece approximation of Chung et al.; below the point
// where that approximation exceeds 1 the check side gives 0.
#include <atomic>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>

#include "internal.hpp"

namespace polarhip {

static thread_local std::string g_last_error;

polar_status set_error(polar_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

polar_status ok_status() {
    g_last_error.clear();
    return POLAR_OK;
}

polar_status hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return POLAR_OK;
    return set_error(POLAR_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int device_cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    static int cached[64] = {0};
    if (dev >= 0 && dev < 64 && cached[dev]) return cached[dev];
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        cus = 256;
    if (dev >= 0 && dev < 64) cached[dev] = cus;
    return cus;
}

// ---------------------------------------------------------------- GA

namespace {

// natural log of the Chung et al. approximation of phi
double ln_phi(double x) {
    if (x <= 0.0) return 0.0;
    if (x < 10.0) return 0.0218 - 0.4527 * std::pow(x, 0.86);
    return -0.25 * x + 0.5 * std::log(M_PI / x) + std::log1p(-10.0 / (7.0 * x));
}

// inverse of ln_phi: smallest x with ln_phi(x) <= t (t <= 0)
double ln_phi_inverse(double t) {
    const double edge = 0.0218 - 0.4527 * std::pow(10.0, 0.86);
    if (t >= 0.0) return 0.0;
    if (t >= edge) return std::pow((0.0218 - t) / 0.4527, 1.0 / 0.86);
    // x >= 10: ln_phi strictly decreasing; Newton from the asymptote, then a
    // bracketing safeguard
    double lo = 10.0, hi = std::max(20.0, -8.0 * t + 40.0);
    while (ln_phi(hi) > t) hi *= 2.0;
    double x = std::min(std::max(-4.0 * t, lo), hi);
    for (int it = 0; it < 100; ++it) {
        double f = ln_phi(x) - t;
        if (f > 0) lo = x; else hi = x;
        double d = -0.25 - 0.5 / x + (10.0 / (7.0 * x * x)) / (1.0 - 10.0 / (7.0 * x));
        double xn = x - f / d;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (std::fabs(xn - x) <= 1e-15 * x) {
            x = xn;
            break;
        }
        x = xn;
    }
    return x;
}

std::vector<double> ga_bit_channel_means(int n, double sigma2) {
    std::vector<double> m(1, 2.0 / sigma2);
    for (int step = 0; step < n; ++step) {
        std::vector<double> nx(m.size() * 2);
        for (size_t q = 0; q < m.size(); ++q) {
            double lp = ln_phi(m[q]);
            double p = std::exp(lp);
            nx[2 * q] = ln_phi_inverse(lp + std::log(2.0 - p));  // check side
            nx[2 * q + 1] = 2.0 * m[q];                          // variable side
        }
        m.swap(nx);
    }
    return m;
}

uint32_t default_poly(int c) {
    switch (c) {
        case 8: return 0x07u;
        case 16: return 0x1021u;
        case 24: return 0x864CFBu;
        default: return 0u;
    }
}

// CRC register after feeding a single 1 followed by `zeros` zero bits
// (shift register, most significant bit first, zero initial state).
uint32_t crc_of_single_one(uint32_t poly, int c, int zeros) {
    const uint32_t mask = (c == 32) ? 0xffffffffu : ((1u << c) - 1u);
    const uint32_t top = 1u << (c - 1);
    uint32_t reg = poly & mask;  // the 1 enters with an empty register
    for (int z = 0; z < zeros; ++z) {
        bool fb = (reg & top) != 0;
        reg = (reg << 1) & mask;
        if (fb) reg ^= poly;
    }
    return reg;
}

template <typename T>
polar_status upload(T** dst, const std::vector<T>& src) {
    size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
    hipError_t e = hipMalloc((void**)dst, bytes);
    if (e != hipSuccess)
        return set_error(POLAR_ERR_NO_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
    if (!src.empty()) {
        e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_check(e, "hipMemcpy");
    }
    return POLAR_OK;
}

}  // namespace
}  // namespace polarhip

using namespace polarhip;

extern "C" {

const char* polar_last_error(void) { return g_last_error.c_str(); }

void polar_free_code(polar_code* code) {
    if (!code) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(code->device);
    (void)hipFree(code->d_frozen_bits);
    (void)hipFree(code->d_info_pos);
    (void)hipFree(code->d_syn);
    (void)hipFree(code->d_syn_nib);
    (void)hipFree(code->d_enc_crc);
    (void)hipFree(code->d_da_bits);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete code;
}

static polar_status validate_sizes(int N, int K, int c) {
    if (N < 8 || N > 4096 || (N & (N - 1)) != 0)
        return set_error(POLAR_ERR_INVALID_ARG, "N must be a power of two in [8, 4096]");
    if (!(c == 0 || c == 8 || c == 16 || c == 24))
        return set_error(POLAR_ERR_INVALID_ARG, "crc_bits must be 0, 8, 16 or 24");
    if (K < 1 || K + c > N) return set_error(POLAR_ERR_INVALID_ARG, "need 1 <= K and K + crc_bits <= N");
    return POLAR_OK;
}

// positions ordered from the most reliable (Gaussian approximation at the
// design point, rate K/N); equal means: higher index first
static std::vector<int> reliability_order(int N, int K, double design_ebn0_db) {
    int n = 0;
    while ((1 << n) < N) ++n;
    const double rate = double(K) / double(N);
    const double sigma2 = 1.0 / (2.0 * rate * std::pow(10.0, design_ebn0_db / 10.0));
    std::vector<double> m = ga_bit_channel_means(n, sigma2);
    std::vector<int> order(N);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (m[a] != m[b]) return m[a] > m[b];
        return a > b;
    });
    return order;
}

static void ga_frozen_mask(int N, int K, int c, double design_ebn0_db, uint8_t* frozen) {
    const std::vector<int> order = reliability_order(N, K, design_ebn0_db);
    for (int i = 0; i < N; ++i) frozen[i] = 1;
    for (int q = 0; q < K + c; ++q) frozen[order[q]] = 0;
}

polar_status polar_construct_frozen(int32_t N, int32_t K, int32_t crc_bits, double design_ebn0_db,
                                    uint8_t* host_mask) {
    if (!host_mask) return set_error(POLAR_ERR_INVALID_ARG, "polar_construct_frozen: null mask");
    polar_status st = validate_sizes(N, K, crc_bits);
    if (st != POLAR_OK) return st;
    ga_frozen_mask(N, K, crc_bits, design_ebn0_db, host_mask);
    return ok_status();
}

polar_status polar_build_code(const polar_code_desc* d, polar_code** out) {
    if (!d || !out) return set_error(POLAR_ERR_INVALID_ARG, "polar_build_code: null argument");
    *out = nullptr;
    const int N = d->N, K = d->K, c = d->crc_bits;
    polar_status vst = validate_sizes(N, K, c);
    if (vst != POLAR_OK) return vst;
    uint32_t poly = c ? (d->crc_poly ? d->crc_poly : default_poly(c)) : 0u;
    if (c && (poly >> c) != 0) return set_error(POLAR_ERR_INVALID_ARG, "crc_poly wider than crc_bits");
    const int k = K + c;
    int n = 0;
    while ((1 << n) < N) ++n;

    std::vector<uint8_t> frozen(N, 1);
    if (d->frozen) {
        int ones = 0;
        for (int i = 0; i < N; ++i) {
            if (d->frozen[i] > 1) return set_error(POLAR_ERR_INVALID_ARG, "frozen mask entries must be 0/1");
            frozen[i] = d->frozen[i];
            ones += frozen[i];
        }
        if (ones != N - k)
            return set_error(POLAR_ERR_INVALID_ARG, "frozen mask must freeze exactly N - K - crc_bits positions");
    } else {
        ga_frozen_mask(N, K, c, d->design_ebn0_db, frozen.data());
    }
    if (d->da_bits < 0 || d->da_bits > k)
        return set_error(POLAR_ERR_INVALID_ARG, "da_bits must be in [0, K + crc_bits]");
    std::vector<uint8_t> da(N, 0);
    if (d->da_bits > 0) {
        const std::vector<int> order = reliability_order(N, K, d->design_ebn0_db);
        int taken = 0;
        for (int q = 0; q < N && taken < d->da_bits; ++q)
            if (!frozen[order[q]]) {
                da[order[q]] = 1;
                ++taken;
            }
    }

    static std::atomic<uint64_t> next_serial{1};
    polar_code* code = new polar_code();
    code->serial = next_serial.fetch_add(1);
    code->N = N;
    code->n = n;
    code->K = K;
    code->c = c;
    code->k = k;
    code->poly = poly;
    code->frozen = frozen;
    code->da = da;
    (void)hipGetDevice(&code->device);
    for (int i = 0; i < N; ++i)
        if (!frozen[i]) code->info_pos.push_back((int16_t)i);

    // tables
    std::vector<uint32_t> fbits(std::max(N / 32, 1), 0u);
    for (int i = 0; i < N; ++i)
        if (frozen[i]) fbits[i / 32] |= 1u << (i % 32);
    std::vector<uint32_t> dbits(std::max(N / 32, 1), 0u);
    for (int i = 0; i < N; ++i)
        if (da[i]) dbits[i / 32] |= 1u << (i % 32);
    std::vector<uint32_t> enc(K, 0u);
    if (c)
        for (int q = 0; q < K; ++q) enc[q] = crc_of_single_one(poly, c, K - 1 - q);
    std::vector<uint32_t> syn(N, 0u);
    if (c) {
        for (int q = 0; q < K; ++q) syn[code->info_pos[q]] = enc[q];
        for (int j = 0; j < c; ++j) syn[code->info_pos[K + j]] = 1u << (c - 1 - j);
    }
    std::vector<uint32_t> nib((size_t)(N / 4) * 16, 0u);
    for (int g = 0; g < N / 4; ++g)
        for (int v = 0; v < 16; ++v) {
            uint32_t s = 0;
            for (int b = 0; b < 4; ++b)
                if (v & (1 << b)) s ^= syn[4 * g + b];
            nib[(size_t)g * 16 + v] = s;
        }
    polar_status st;
    if ((st = upload(&code->d_frozen_bits, fbits)) != POLAR_OK ||
        (st = upload(&code->d_info_pos, code->info_pos)) != POLAR_OK ||
        (st = upload(&code->d_syn, syn)) != POLAR_OK ||
        (st = upload(&code->d_syn_nib, nib)) != POLAR_OK ||
        (st = upload(&code->d_enc_crc, enc)) != POLAR_OK ||
        (st = upload(&code->d_da_bits, dbits)) != POLAR_OK) {
        polar_free_code(code);
        return st;
    }
    *out = code;
    return ok_status();
}

polar_status polar_code_params(const polar_code* code, int32_t* N, int32_t* K, int32_t* crc_bits,
                               uint32_t* crc_poly) {
    if (!code) return set_error(POLAR_ERR_INVALID_ARG, "polar_code_params: null code");
    if (N) *N = code->N;
    if (K) *K = code->K;
    if (crc_bits) *crc_bits = code->c;
    if (crc_poly) *crc_poly = code->poly;
    return ok_status();
}

polar_status polar_code_frozen(const polar_code* code, uint8_t* host_mask) {
    if (!code || !host_mask) return set_error(POLAR_ERR_INVALID_ARG, "polar_code_frozen: null argument");
    std::memcpy(host_mask, code->frozen.data(), code->N);
    return ok_status();
}

polar_status polar_code_decision_aided(const polar_code* code, uint8_t* host_mask) {
    if (!code || !host_mask) return set_error(POLAR_ERR_INVALID_ARG, "polar_code_decision_aided: null argument");
    std::memcpy(host_mask, code->da.data(), code->N);
    return ok_status();
}

}  // extern "C"

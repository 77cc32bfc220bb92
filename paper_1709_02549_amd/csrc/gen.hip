// GPU generator of seeded synthetic scans (planar recipes: one tumour and
// clutter point scatterers in a disc, homogeneous medium, white noise).  It
// produces the training scans of the learned proposer without a host round trip
// and follows the host generator's definition draw for draw:
//   * scene: SplitMix64 (Steele, Lea, Flood 2014) seeded with seed ^ (salt << 56):
//     tumour (r = R sqrt(u), theta = 2 pi u'), then every clutter point the same
//     way, then the clutter reflectivities rho = 0.1 u (each draw taken directly
//     from its index, one scatterer per lane);
//   * echoes: Y_i[n] = sum_s A_is p(t0 + n dt - 2 |x_s - a_i| / v),
//     A_is = rho_s (1 cm / |x_s - a_i|)^2,
//     p(t) = sin(2 pi f0 t) exp(-t^2 / 2 sigma^2) / peak for |t| <= 6 sigma;
//   * noise: sigma_n^2 = P / 10^(SNR/10), P = mean over antennas of the tumour
//     echo's mean square over samples within 3 sigma of its arrival; N(0,1)
//     deviates from Philox4x32-10 (Salmon et al. 2011), counter (sample pair,
//     antenna, tag, 0), key (seed low, seed high), Box-Muller (cosine for the even
//     sample, sine for the odd one).
// One workgroup per (scan, antenna); each lane owns 8 consecutive samples and adds
// every scatterer's contribution in scatterer order, so the result is deterministic.
#include <cmath>

#include "uwb_internal.h"

namespace uwb {
namespace {

constexpr int kMaxScat = 1024;   // scatterers per scene (LDS: 40 B each)
constexpr uint32_t kNoiseTag = 0x4E4F4953u;

// SplitMix64 adds a constant to its state before every output, so draw d (0-based)
// of a stream seeded with s0 is the output mix of s0 + (d + 1) * gamma: any draw can
// be taken directly, and the scatterers of a scene are drawn in parallel.
__device__ __forceinline__ double splitmix_uniform(unsigned long long s0, unsigned long long d) {
    unsigned long long z = s0 + (d + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

__device__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const unsigned long long p0 = (unsigned long long)0xD2511F53u * c[0];
        const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
}

struct GenArgs {
    const float *ant_pos;   // [M][3]
    const unsigned long long *seeds;
    float *traces;          // [n][M][T]
    double *tumours;        // [n][3] or null
    int M, T, n_clutter;
    double v, dt, t0, radius, snr_db, f0, sigma, peak;
    unsigned long long salt;
};

__device__ __forceinline__ float pulse32(float t, float f0, float sigma, float inv_peak) {
    if (fabsf(t) > 6.f * sigma) return 0.f;
    return sinf(6.283185307179586f * f0 * t) * expf(-(t * t) / (2.f * sigma * sigma)) * inv_peak;
}

// One workgroup per (scan, antenna): every workgroup of a scan redraws the (cheap)
// scene and the tumour power, then synthesises its antenna's trace.
// Dynamic LDS: scene and per-scatterer terms for ns scatterers, then the reduction space.
__host__ __device__ inline size_t gen_lds_bytes(int ns) { return (size_t)ns * (4 * sizeof(double) + 8) + 256 * 16; }

__global__ __launch_bounds__(256) void k_gen_disc(const GenArgs a) {
    extern __shared__ __align__(16) unsigned char gsm[];
    const int ns = a.n_clutter + 1;
    double *sx = reinterpret_cast<double *>(gsm), *sy = sx + ns, *srho = sy + ns, *s_tau = srho + ns;
    float *s_amp = reinterpret_cast<float *>(s_tau + ns);
    int *s_n0 = reinterpret_cast<int *>(s_amp + ns);
    double *red = reinterpret_cast<double *>(gsm + (((size_t)ns * (4 * sizeof(double) + 8) + 15) & ~(size_t)15));
    int *redn = reinterpret_cast<int *>(red + 256);
    const int scan = blockIdx.x, i = blockIdx.y, tid = threadIdx.x;
    const unsigned long long seed = a.seeds[scan];
    // scene: scatterer s takes draws 2 s (radius) and 2 s + 1 (angle); clutter point
    // s >= 1 its reflectivity from draw 2 ns + s - 1, after every position
    const unsigned long long s0 = seed ^ (a.salt << 56);
    for (int s = tid; s < ns; s += 256) {
        const double rr = a.radius * sqrt(splitmix_uniform(s0, 2ull * s));
        const double th = 2.0 * M_PI * splitmix_uniform(s0, 2ull * s + 1);
        sx[s] = rr * cos(th);
        sy[s] = rr * sin(th);
        srho[s] = s == 0 ? 1.0 : 0.1 * splitmix_uniform(s0, 2ull * ns + s - 1);
    }
    __syncthreads();
    if (a.tumours && i == 0 && tid == 0) {
        a.tumours[3 * scan + 0] = sx[0];
        a.tumours[3 * scan + 1] = sy[0];
        a.tumours[3 * scan + 2] = 0.0;
    }
    const float sigma = (float)a.sigma, f0 = (float)a.f0, inv_peak = (float)(1.0 / a.peak);
    const double half = 6.0 * a.sigma;
    // tumour echo power: mean over antennas of its mean square within 3 sigma of arrival.
    // G threads per antenna (G = 256 / M rounded down to a power of two, at least 1) take
    // every G-th sample of its window; the parts are added in thread order.
    int G = 1;
    while (2 * G * a.M <= 256) G *= 2;
    const int per = 256 / G;   // antennas per pass
    double pw = 0.0;
    for (int k0 = 0; k0 < a.M; k0 += per) {
        const int k = k0 + tid / G, g = tid % G;
        double sq = 0.0;
        int cnt = 0;
        if (k < a.M) {
            const double ax = a.ant_pos[3 * k], ay = a.ant_pos[3 * k + 1], az = a.ant_pos[3 * k + 2];
            const double dx = sx[0] - ax, dy = sy[0] - ay, dz = -az;
            const double dist = sqrt(dx * dx + dy * dy + dz * dz);
            const double tau = 2.0 * dist / a.v;
            const double amp = (0.01 / dist) * (0.01 / dist);
            const long long lo = (long long)ceil((tau - 3.0 * a.sigma - a.t0) / a.dt);
            const long long hi = (long long)floor((tau + 3.0 * a.sigma - a.t0) / a.dt);
            for (long long m = lo - 1 + g; m <= hi + 1; m += G) {
                if (m < 0 || m >= a.T) continue;
                const double t = a.t0 + m * a.dt - tau;
                if (fabs(t) > 3.0 * a.sigma) continue;
                const double p = fabs(t) <= half
                                     ? amp * sin(2.0 * M_PI * a.f0 * t) * exp(-(t * t) / (2.0 * a.sigma * a.sigma)) / a.peak
                                     : 0.0;
                sq += p * p;
                ++cnt;
            }
        }
        __syncthreads();   // the previous pass's parts are consumed
        red[tid] = sq;
        redn[tid] = cnt;
        __syncthreads();
        if (g == 0 && k < a.M) {
            double sk = 0.0;
            int ck = 0;
            for (int j = 0; j < G; ++j) { sk += red[tid + j]; ck += redn[tid + j]; }
            red[tid] = ck ? sk / ck : 0.0;   // this antenna's mean square
        }
        __syncthreads();
        if (tid == 0)
            for (int kk = k0; kk < a.M && kk < k0 + per; ++kk) pw += red[(kk - k0) * G];
    }
    __syncthreads();
    if (tid == 0) red[0] = pw;
    __syncthreads();
    const double ps = red[0] / a.M;
    const double sigma_n = sqrt(ps / pow(10.0, a.snr_db / 10.0));
    // this workgroup's antenna
    const double ax = a.ant_pos[3 * i], ay = a.ant_pos[3 * i + 1], az = a.ant_pos[3 * i + 2];
    for (int s = tid; s < ns; s += 256) {
        const double dx = sx[s] - ax, dy = sy[s] - ay, dz = -az;
        const double dist = sqrt(dx * dx + dy * dy + dz * dz);
        const double tau = 2.0 * dist / a.v;
        s_tau[s] = tau - a.t0;
        s_amp[s] = (float)(srho[s] * (0.01 / dist) * (0.01 / dist));
        s_n0[s] = (int)floor((tau - half - a.t0) / a.dt);
    }
    __syncthreads();
    float acc[8];
    const int m0 = tid * 8;
    for (int q = 0; q < 8; ++q) acc[q] = 0.f;
    if (m0 < a.T) {
        for (int s = 0; s < ns; ++s) {
            const int n0 = s_n0[s];
            if (n0 + 40 < m0 || n0 > m0 + 7) continue;
            const double tau = s_tau[s];
            const float amp = s_amp[s];
            for (int q = 0; q < 8; ++q) {
                const float t = (float)((double)(m0 + q) * a.dt - tau);   // difference in FP64, pulse in FP32
                acc[q] += amp * pulse32(t, f0, sigma, inv_peak);
            }
        }
        // noise: pairs (m0/2 .. m0/2 + 3) of this antenna
        for (int pq = 0; pq < 4; ++pq) {
            uint32_t c[4] = {(uint32_t)(m0 / 2 + pq), (uint32_t)i, kNoiseTag, 0u};
            philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
            const double u1 = ((double)c[0] + 0.5) * (1.0 / 4294967296.0);
            const double u2 = ((double)c[1] + 0.5) * (1.0 / 4294967296.0);
            const double rr = sqrt(-2.0 * log(u1));
            acc[2 * pq] = (float)((double)acc[2 * pq] + sigma_n * rr * cos(2.0 * M_PI * u2));
            acc[2 * pq + 1] = (float)((double)acc[2 * pq + 1] + sigma_n * rr * sin(2.0 * M_PI * u2));
        }
        float *out = a.traces + ((size_t)scan * a.M + i) * a.T;
        for (int q = 0; q < 8; ++q)
            if (m0 + q < a.T) out[m0 + q] = acc[q];
    }
}

}  // namespace
}  // namespace uwb

using namespace uwb;

extern "C" int uwb_generate_disc_scans(const uwb_gen_recipe *r, const float *ant_pos, const uint64_t *seeds,
                                       int32_t n, float *traces, double *tumours, void *stream) {
    if (!r || !ant_pos || !seeds || !traces || n < 1) return UWB_EINVAL;
    if (r->n_ant < 1 || r->n_samp < 2 || r->n_clutter < 0) return UWB_EINVAL;
    if (r->n_clutter + 1 > kMaxScat || r->n_samp > 256 * 8 * 16) return UWB_EUNSUPPORTED;
    const double vals[8] = {r->v, r->dt, r->radius, r->pulse_f0, r->pulse_sigma, r->pulse_peak, r->t0, r->snr_db};
    for (double x : vals)
        if (!std::isfinite(x)) return UWB_EINVAL;
    if (!(r->v > 0 && r->dt > 0 && r->radius > 0 && r->pulse_sigma > 0 && r->pulse_peak > 0)) return UWB_EINVAL;
    if (r->n_samp > 2048 * 8) return UWB_EUNSUPPORTED;
    if (n > 0x7fffffff) return UWB_EUNSUPPORTED;
    GenArgs a;
    a.ant_pos = ant_pos;
    a.seeds = reinterpret_cast<const unsigned long long *>(seeds);
    a.traces = traces;
    a.tumours = tumours;
    a.M = r->n_ant;
    a.T = r->n_samp;
    a.n_clutter = r->n_clutter;
    a.v = r->v;
    a.dt = r->dt;
    a.t0 = r->t0;
    a.radius = r->radius;
    a.snr_db = r->snr_db;
    a.f0 = r->pulse_f0;
    a.sigma = r->pulse_sigma;
    a.peak = r->pulse_peak;
    a.salt = r->salt;
    if (a.T > 256 * 8) return UWB_EUNSUPPORTED;   // one pass of 8 samples per lane
    if (a.M > 65535) return UWB_EUNSUPPORTED;
    hipLaunchKernelGGL(k_gen_disc, dim3(n, a.M), dim3(256), gen_lds_bytes(a.n_clutter + 1), (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? UWB_OK : UWB_EHIP;
}

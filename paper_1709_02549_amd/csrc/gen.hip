// GPU generator of seeded synthetic scans (planar recipes: one tumour and
// clutter point scatterers in a disc, homogeneous medium, white noise).  It
// produces the training scans of the learned proposer without a host round trip
// and follows the host generator's definition draw for draw:
//   * scene: SplitMix64 (Steele, Lea, Flood 2014) seeded with seed ^ (salt << 56):
//     tumour (r = R sqrt(u), theta = 2 pi u'), then every clutter point the same
//     way, then the clutter reflectivities rho = 0.1 u;
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

constexpr int kMaxScat = 1024;
constexpr uint32_t kNoiseTag = 0x4E4F4953u;

struct SplitMix64 {
    unsigned long long s;
    __device__ unsigned long long next() {
        s += 0x9E3779B97F4A7C15ull;
        unsigned long long z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    __device__ double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

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
__global__ __launch_bounds__(256) void k_gen_disc(const GenArgs a) {
    __shared__ double sx[kMaxScat + 1], sy[kMaxScat + 1], srho[kMaxScat + 1];
    __shared__ double s_tau[kMaxScat + 1];
    __shared__ float s_amp[kMaxScat + 1];
    __shared__ int s_n0[kMaxScat + 1];
    __shared__ double red[256];
    const int scan = blockIdx.x, i = blockIdx.y, tid = threadIdx.x;
    const unsigned long long seed = a.seeds[scan];
    const int ns = a.n_clutter + 1;
    if (tid == 0) {
        SplitMix64 r{seed ^ (a.salt << 56)};
        for (int s = 0; s < ns; ++s) {
            const double rr = a.radius * sqrt(r.uniform());
            const double th = 2.0 * M_PI * r.uniform();
            sx[s] = rr * cos(th);
            sy[s] = rr * sin(th);
        }
        srho[0] = 1.0;
        for (int s = 1; s < ns; ++s) srho[s] = 0.1 * r.uniform();
        if (a.tumours && i == 0) {
            a.tumours[3 * scan + 0] = sx[0];
            a.tumours[3 * scan + 1] = sy[0];
            a.tumours[3 * scan + 2] = 0.0;
        }
    }
    __syncthreads();
    const float sigma = (float)a.sigma, f0 = (float)a.f0, inv_peak = (float)(1.0 / a.peak);
    const double half = 6.0 * a.sigma;
    // tumour echo power: mean over antennas of its mean square within 3 sigma of arrival
    double pw = 0.0;
    for (int k = tid; k < a.M; k += 256) {
        const double ax = a.ant_pos[3 * k], ay = a.ant_pos[3 * k + 1], az = a.ant_pos[3 * k + 2];
        const double dx = sx[0] - ax, dy = sy[0] - ay, dz = -az;
        const double dist = sqrt(dx * dx + dy * dy + dz * dz);
        const double tau = 2.0 * dist / a.v;
        const double amp = (0.01 / dist) * (0.01 / dist);
        double sq = 0.0;
        int cnt = 0;
        const long long lo = (long long)ceil((tau - 3.0 * a.sigma - a.t0) / a.dt);
        const long long hi = (long long)floor((tau + 3.0 * a.sigma - a.t0) / a.dt);
        for (long long m = lo - 1; m <= hi + 1; ++m) {
            if (m < 0 || m >= a.T) continue;
            const double t = a.t0 + m * a.dt - tau;
            if (fabs(t) > 3.0 * a.sigma) continue;
            const double p = fabs(t) <= half
                                 ? amp * sin(2.0 * M_PI * a.f0 * t) * exp(-(t * t) / (2.0 * a.sigma * a.sigma)) / a.peak
                                 : 0.0;
            sq += p * p;
            ++cnt;
        }
        pw += cnt ? sq / cnt : 0.0;
    }
    red[tid] = pw;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
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
    hipLaunchKernelGGL(k_gen_disc, dim3(n, a.M), dim3(256), 0, (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? UWB_OK : UWB_EHIP;
}

/*
 * FP64 reference ("oracle") for DAS and DMAS confocal imaging.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It is deliberately plain and
 * slow: every quantity is computed straight from its definition, in double
 * precision, with no tiling, no reuse across voxels and no regrouping of sums.
 * It shares no source, header or constant with the GPU library.
 *
 * The method (Section II of the paper):
 *   delay      Eq. (1), read as the monostatic round trip in samples,
 *              n_i(r) = (2 |r - a_i| / v - t0) / dt
 *              (the printed equation divides by 2 c dt; Eq. (2) with the
 *              transmitter equal to the receiver shows the factor 2 multiplies
 *              the path length, and v is the speed in the medium).
 *   alignment  Eq. (3) argument: the trace is advanced by the delay, so the echo
 *              of a scatterer at r lands at window offset k = 0 for every antenna.
 *              Fractional delays use linear interpolation; samples outside [0,T)
 *              are zero.
 *   DAS        Eq. (3): I(r) = sum_k ( sum_i s_i(r,k) )^2 over a centred window
 *              k = -h..h of W = 2h+1 samples.
 *   DMAS       Section II-B (the figure with its equation is not available):
 *              every pair of aligned signals is multiplied and the products are
 *              summed, then the windowed energy is taken:
 *              I(r) = sum_k ( sum_{i<j} s_i(r,k) s_j(r,k) )^2.
 *              Evaluated here as the literal O(M^2) double loop.
 *   samples    The aligned window samples themselves are exported too, for the
 *              Capon (MVDR) beamformer of oracle/mvdr.py, which weights them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Y_i[m] with zero outside the recorded samples. */
static double sample_or_zero(const float *trace, int n_samp, long m)
{
    if (m < 0 || m >= n_samp)
        return 0.0;
    return (double)trace[m];
}

/* Eq. (1) (monostatic round trip, reading above), in samples. */
static double round_trip_delay(const double r[3], const float *a, double v, double dt, double t0)
{
    double dx = r[0] - (double)a[0];
    double dy = r[1] - (double)a[1];
    double dz = r[2] - (double)a[2];
    double dist = sqrt(dx * dx + dy * dy + dz * dz);
    return (2.0 * dist / v - t0) / dt;
}

/* Eq. (3) argument: trace value at fractional position tau + k, linear interpolation. */
static double aligned_sample(const float *trace, int n_samp, double tau, int k)
{
    double x = tau + (double)k;
    double n = floor(x);
    double f = x - n;
    long m = (long)n;
    return (1.0 - f) * sample_or_zero(trace, n_samp, m) + f * sample_or_zero(trace, n_samp, m + 1);
}

/* Energy of one focal point. beamformer: 0 = DAS (Eq. 3), 1 = DMAS (direct pairwise). */
static double focal_point_energy(int beamformer, int n_ant, int n_samp, const float *ant_pos,
                                 const float *traces, double dt, double t0, double v, int window,
                                 const double r[3], double *tau, double *s)
{
    int h = (window - 1) / 2;
    for (int i = 0; i < n_ant; ++i)
        tau[i] = round_trip_delay(r, ant_pos + 3 * i, v, dt, t0);
    double energy = 0.0;
    for (int k = -h; k <= h; ++k) {
        for (int i = 0; i < n_ant; ++i)
            s[i] = aligned_sample(traces + (size_t)i * n_samp, n_samp, tau[i], k);
        double sum;
        if (beamformer == 0) {
            sum = 0.0;
            for (int i = 0; i < n_ant; ++i)
                sum += s[i];
        } else {
            sum = 0.0;
            for (int i = 0; i < n_ant - 1; ++i)
                for (int j = i + 1; j < n_ant; ++j)
                    sum += s[i] * s[j];
        }
        energy += sum * sum;
    }
    return energy;
}

/*
 * Image an explicit list of voxels of a grid.
 *   idx    [n][3] int32 voxel indices (ix, iy, iz); position = origin + idx * pitch
 *   out    [n] energies
 *   n_threads  OpenMP threads (<= 0: library default).  Returns the count used.
 */
int oracle_image_indices(int beamformer, int n_ant, int n_samp, const float *ant_pos,
                         const float *traces, double dt, double t0, double v, int window,
                         const double *origin, const double *pitch, long n, const int32_t *idx,
                         double *out, int n_threads)
{
    int used = 1;
#ifdef _OPENMP
    if (n_threads <= 0)
        n_threads = omp_get_max_threads();
    used = n_threads;
#pragma omp parallel num_threads(n_threads)
#endif
    {
        double *tau = (double *)malloc(sizeof(double) * (size_t)n_ant);
        double *s = (double *)malloc(sizeof(double) * (size_t)n_ant);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
        for (long p = 0; p < n; ++p) {
            double r[3];
            for (int d = 0; d < 3; ++d)
                r[d] = origin[d] + (double)idx[3 * p + d] * pitch[d];
            out[p] = focal_point_energy(beamformer, n_ant, n_samp, ant_pos, traces, dt, t0, v,
                                        window, r, tau, s);
        }
        free(tau);
        free(s);
    }
    return used;
}

/*
 * The aligned window samples themselves, for beamformers that weight them
 * (Capon / MVDR): out[p][i][k + h] = s_i(r_p, k), the Eq. (3) argument of
 * antenna i at window offset k = -h..h, linear interpolation, zero outside the
 * trace.  out holds n * n_ant * window doubles.
 */
int oracle_aligned_samples(int n_ant, int n_samp, const float *ant_pos, const float *traces, double dt,
                           double t0, double v, int window, const double *origin, const double *pitch, long n,
                           const int32_t *idx, double *out, int n_threads)
{
    int used = 1;
    int h = (window - 1) / 2;
#ifdef _OPENMP
    if (n_threads <= 0)
        n_threads = omp_get_max_threads();
    used = n_threads;
#pragma omp parallel for num_threads(n_threads) schedule(dynamic, 64)
#endif
    for (long p = 0; p < n; ++p) {
        double r[3];
        for (int d = 0; d < 3; ++d)
            r[d] = origin[d] + (double)idx[3 * p + d] * pitch[d];
        for (int i = 0; i < n_ant; ++i) {
            double tau = round_trip_delay(r, ant_pos + 3 * i, v, dt, t0);
            for (int k = -h; k <= h; ++k)
                out[((size_t)p * n_ant + i) * window + (k + h)] =
                    aligned_sample(traces + (size_t)i * n_samp, n_samp, tau, k);
        }
    }
    return used;
}

/*
 * Multistatic imaging (Eq. (2) and Eq. (4)): every antenna transmits and every
 * antenna receives, giving M^2 channels Y_ij, traces[(i*M + j)*n_samp ...].
 *   delay      Eq. (2): the transmitter-to-point plus point-to-receiver path,
 *              n_ij(r) = ((|r - a_i| + |r - a_j|) / v - t0) / dt
 *              (with i = j this is the monostatic delay above).
 *   DAS        Eq. (4): I(r) = sum_k ( sum_i sum_j s_ij(r,k) )^2, all M^2 channels.
 *   DMAS       Section II-B applied to the M^2 channel signals: the sum over every
 *              pair of distinct channels of the product of their aligned samples,
 *              then the windowed energy (literal double loop over channel pairs).
 */
static double path_delay(const double r[3], const float *a_tx, const float *a_rx, double v, double dt,
                         double t0)
{
    double d_tx = 0.0, d_rx = 0.0;
    for (int d = 0; d < 3; ++d) {
        double u = r[d] - (double)a_tx[d];
        double w = r[d] - (double)a_rx[d];
        d_tx += u * u;
        d_rx += w * w;
    }
    return ((sqrt(d_tx) + sqrt(d_rx)) / v - t0) / dt;
}

static double focal_point_energy_ms(int beamformer, int n_ant, int n_samp, const float *ant_pos,
                                    const float *traces, double dt, double t0, double v, int window,
                                    const double r[3], double *tau, double *s)
{
    int h = (window - 1) / 2;
    int n_ch = n_ant * n_ant;
    for (int i = 0; i < n_ant; ++i)
        for (int j = 0; j < n_ant; ++j)
            tau[i * n_ant + j] = path_delay(r, ant_pos + 3 * i, ant_pos + 3 * j, v, dt, t0);
    double energy = 0.0;
    for (int k = -h; k <= h; ++k) {
        for (int c = 0; c < n_ch; ++c)
            s[c] = aligned_sample(traces + (size_t)c * n_samp, n_samp, tau[c], k);
        double sum = 0.0;
        if (beamformer == 0) {
            for (int c = 0; c < n_ch; ++c)
                sum += s[c];
        } else {
            for (int c = 0; c < n_ch - 1; ++c)
                for (int e = c + 1; e < n_ch; ++e)
                    sum += s[c] * s[e];
        }
        energy += sum * sum;
    }
    return energy;
}

/* Multistatic counterpart of oracle_image_indices: n_ant = M antennas, M^2 traces. */
int oracle_image_indices_ms(int beamformer, int n_ant, int n_samp, const float *ant_pos,
                            const float *traces, double dt, double t0, double v, int window,
                            const double *origin, const double *pitch, long n, const int32_t *idx,
                            double *out, int n_threads)
{
    int used = 1;
#ifdef _OPENMP
    if (n_threads <= 0)
        n_threads = omp_get_max_threads();
    used = n_threads;
#pragma omp parallel num_threads(n_threads)
#endif
    {
        size_t n_ch = (size_t)n_ant * (size_t)n_ant;
        double *tau = (double *)malloc(sizeof(double) * n_ch);
        double *s = (double *)malloc(sizeof(double) * n_ch);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (long p = 0; p < n; ++p) {
            double r[3];
            for (int d = 0; d < 3; ++d)
                r[d] = origin[d] + (double)idx[3 * p + d] * pitch[d];
            out[p] = focal_point_energy_ms(beamformer, n_ant, n_samp, ant_pos, traces, dt, t0, v,
                                           window, r, tau, s);
        }
        free(tau);
        free(s);
    }
    return used;
}

/* Multistatic counterpart of oracle_aligned_samples: the M^2 channels (Eq. (2) delay), out [n][M*M][window]. */
int oracle_aligned_samples_ms(int n_ant, int n_samp, const float *ant_pos, const float *traces, double dt,
                              double t0, double v, int window, const double *origin, const double *pitch, long n,
                              const int32_t *idx, double *out, int n_threads)
{
    int used = 1;
    int h = (window - 1) / 2;
    size_t n_ch = (size_t)n_ant * (size_t)n_ant;
#ifdef _OPENMP
    if (n_threads <= 0)
        n_threads = omp_get_max_threads();
    used = n_threads;
#pragma omp parallel for num_threads(n_threads) schedule(dynamic, 16)
#endif
    for (long p = 0; p < n; ++p) {
        double r[3];
        for (int d = 0; d < 3; ++d)
            r[d] = origin[d] + (double)idx[3 * p + d] * pitch[d];
        for (int i = 0; i < n_ant; ++i)
            for (int j = 0; j < n_ant; ++j) {
                size_t c = (size_t)i * n_ant + j;
                double tau = path_delay(r, ant_pos + 3 * i, ant_pos + 3 * j, v, dt, t0);
                for (int k = -h; k <= h; ++k)
                    out[((size_t)p * n_ch + c) * window + (k + h)] =
                        aligned_sample(traces + c * n_samp, n_samp, tau, k);
            }
    }
    return used;
}

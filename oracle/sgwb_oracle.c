/*
 * Plain FP64 CPU oracle for folded-data SGWB radiometer map-making
 * (Ain, Suresh & Mitra, "Very fast stochastic gravitational wave background
 * map-making using folded data", arXiv:1803.08285).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links or calls this file;
 * only the tests, the smoke check and the benchmark's CPU-baseline leg do.
 * It shares no code, header, table or constant with the HIP path.
 *
 * Every quantity is computed in double precision with the most direct
 * formula available: explicit polarisation basis for the antenna patterns,
 * libm cos/sin for every (t, f, p) term, sequential sums over segments.
 *
 * Conventions (the paper leaves these open; the readings are listed in the
 * design notes of the repository):
 *   - pixels: HEALPix RING order, centres from the ring formulas of
 *     Gorski et al. (2005), enumerated ring by ring;
 *   - detectors: L-shaped, arms horizontal, x-arm azimuth counter-clockwise
 *     from local East, y-arm at azimuth + 90 deg, response tensor
 *     D = (u u^T - v v^T) / 2, sites on a sphere of radius 6.371e6 m;
 *   - Earth rotation: celestial-frame vector = R_z(theta) * Earth-fixed vector,
 *     theta = 2 pi t / T_s with T_s = 86164.0905 s (one sidereal day, Sec. II.B);
 *   - seeds (Sec. III.D): gamma(t,p) = sum_A F^A_1 F^A_2 at the pixel centre,
 *     tau(t,p) = Omega_p . (x_1(t) - x_2(t)) / c;
 *   - dirty map (Eq. eq_dirtymap, narrowband split Eq. eq:narrowband, constant
 *     prefactors dropped, real part kept):
 *       X(k,p) = sum_t w(t,k) gamma(t,p) Re[ C(t,k) exp(+2 pi i f_k tau(t,p)) ]
 *   - Fisher diagonal per bin (Eq. eq_fisher, diagonal p = p', split per bin as
 *     in Sec. III.A):  G(k,p) = sum_t w(t,k) gamma(t,p)^2
 *   - broadband (Sec. V, spectrum-weighted sum of narrowband maps):
 *       Xbb(p) = sum_k X(k,p),   Gbb(p) = sum_k H(f_k) G(k,p).
 *   - Fisher diagonal with the overlapping-window neighbour terms (Sec. II.B,
 *     Eq. fwGamma with p = p', folded series v, u, w):
 *       G(k,p) = Re sum_t conj(K_t) [K_t v_t - K_{t-1} u_t - K_{t+1} w_t],
 *       K_t = gamma(t,p) exp(+2 pi i f_k tau(t,p)), the day periodic in t;
 *   - folding (Sec. II.B): v, u, w, x summed over days from per-segment CSD C,
 *     inverse variances s = sigma^-2 and presence flags, in absolute time
 *     (the neighbour of a day's first segment is the previous day's last one).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define ORC_EARTH_R 6.371e6
#define ORC_C_LIGHT 299792458.0
#define ORC_T_SID 86164.0905

/* ------------------------------------------------------------------------ */
/* HEALPix RING centres (Sec. III.B; Gorski et al. 2005, ring formulas).      */
/* Walk the 4 nside - 1 iso-latitude rings from north to south.               */
/* ------------------------------------------------------------------------ */
int orc_healpix_centres(int nside, double *xyz)
{
    if (nside < 1) return -1;
    long p = 0;
    const double ns = (double)nside;
    for (int i = 1; i <= 4 * nside - 1; ++i) {
        int npr;          /* pixels in this ring */
        double z;         /* cos(theta) of the ring */
        double shift;     /* phi offset in units of the pixel spacing */
        int north_index = i <= 2 * nside ? i : 4 * nside - i; /* ring index counted from the nearer pole */
        if (north_index < nside) {
            /* polar cap ring */
            npr = 4 * north_index;
            z = 1.0 - (double)north_index * north_index / (3.0 * ns * ns);
            shift = 0.5;
        } else {
            /* equatorial belt ring */
            npr = 4 * nside;
            z = 4.0 / 3.0 - 2.0 * north_index / (3.0 * ns);
            /* rings with i - nside even start half a pixel east of phi = 0,
             * the others start at phi = 0 (reference RING numbering) */
            shift = ((i - nside) % 2 == 0) ? 0.5 : 1.0;
        }
        if (i > 2 * nside) z = -z;
        double sin_theta = sqrt((1.0 - z) * (1.0 + z));
        for (int j = 1; j <= npr; ++j) {
            double phi = (j - shift) * (2.0 * ORC_PI / npr);
            xyz[3 * p + 0] = sin_theta * cos(phi);
            xyz[3 * p + 1] = sin_theta * sin(phi);
            xyz[3 * p + 2] = z;
            ++p;
        }
    }
    return (p == 12L * nside * nside) ? 0 : -2;
}

/* ------------------------------------------------------------------------ */
/* Detector position and response tensor on the Earth-radius sphere.         */
/* ------------------------------------------------------------------------ */
void orc_detector(double lat_deg, double lon_deg, double az_deg, double r[3], double D[9])
{
    const double d2r = ORC_PI / 180.0;
    double la = lat_deg * d2r, lo = lon_deg * d2r, az = az_deg * d2r;
    r[0] = ORC_EARTH_R * cos(la) * cos(lo);
    r[1] = ORC_EARTH_R * cos(la) * sin(lo);
    r[2] = ORC_EARTH_R * sin(la);
    double east[3] = {-sin(lo), cos(lo), 0.0};
    double north[3] = {-sin(la) * cos(lo), -sin(la) * sin(lo), cos(la)};
    double u[3], v[3];
    for (int a = 0; a < 3; ++a) {
        u[a] = cos(az) * east[a] + sin(az) * north[a];
        v[a] = -sin(az) * east[a] + cos(az) * north[a];
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) D[3 * a + b] = 0.5 * (u[a] * u[b] - v[a] * v[b]);
}

/* Antenna patterns F+ and Fx of response tensor D for direction (theta, phi),
 * using the explicit polarisation basis m = (sin phi, -cos phi, 0),
 * n = (cos theta cos phi, cos theta sin phi, -sin theta),
 * e+ = m m^T - n n^T, ex = m n^T + n m^T. */
void orc_antenna(const double D[9], double cos_t, double sin_t, double phi, double *fp, double *fx)
{
    double m[3] = {sin(phi), -cos(phi), 0.0};
    double n[3] = {cos_t * cos(phi), cos_t * sin(phi), -sin_t};
    double sp = 0.0, sx = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double ep = m[a] * m[b] - n[a] * n[b];
            double ex = m[a] * n[b] + n[a] * m[b];
            sp += D[3 * a + b] * ep;
            sx += D[3 * a + b] * ex;
        }
    *fp = sp;
    *fx = sx;
}

/* Rotate a symmetric tensor and a vector about z by angle th:  M' = R M R^T. */
static void rot_z(double th, const double Min[9], const double vin[3], double Mout[9], double vout[3])
{
    double R[9] = {cos(th), -sin(th), 0.0, sin(th), cos(th), 0.0, 0.0, 0.0, 1.0};
    double T[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += R[3 * a + c] * Min[3 * c + b];
            T[3 * a + b] = s;
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += T[3 * a + c] * R[3 * b + c];
            Mout[3 * a + b] = s;
        }
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int c = 0; c < 3; ++c) s += R[3 * a + c] * vin[c];
        vout[a] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* ORF seed matrices (Sec. III.D, Fig. 3): gamma[t][p] and tau[t][p] for all  */
/* pixels, or for the nsel pixels listed in pix (then shape [nt][nsel]).      */
/* det = {latA, lonA, azA, latB, lonB, azB} in degrees.                       */
/* Segment k has mid time t_k = t0 + k*stride + dur/2 (sidereal seconds).     */
/* ------------------------------------------------------------------------ */
int orc_geometry_at(const double det[6], int nside, int nt, double t0, double stride, double dur,
                    long nsel, const int64_t *pix, double *gamma, double *tau)
{
    long npix = 12L * nside * nside;
    double *xyz = (double *)malloc(sizeof(double) * 3 * npix);
    if (!xyz) return -3;
    int rc = orc_healpix_centres(nside, xyz);
    if (rc) { free(xyz); return rc; }
    double rA[3], rB[3], DA[9], DB[9];
    orc_detector(det[0], det[1], det[2], rA, DA);
    orc_detector(det[3], det[4], det[5], rB, DB);
    double dx[3] = {rA[0] - rB[0], rA[1] - rB[1], rA[2] - rB[2]};
    double zero[3] = {0, 0, 0}, dummy[3];
    for (int k = 0; k < nt; ++k) {
        double tk = t0 + k * stride + 0.5 * dur;
        double th = 2.0 * ORC_PI * tk / ORC_T_SID;
        double DAt[9], DBt[9], dxt[3];
        rot_z(th, DA, dx, DAt, dxt);
        rot_z(th, DB, zero, DBt, dummy);
        for (long i = 0; i < nsel; ++i) {
            long p = pix ? (long)pix[i] : i;
            if (p < 0 || p >= npix) { free(xyz); return -4; }
            double ox = xyz[3 * p], oy = xyz[3 * p + 1], oz = xyz[3 * p + 2];
            double sin_t = sqrt(ox * ox + oy * oy);
            double phi = atan2(oy, ox);
            double fpA, fxA, fpB, fxB;
            orc_antenna(DAt, oz, sin_t, phi, &fpA, &fxA);
            orc_antenna(DBt, oz, sin_t, phi, &fpB, &fxB);
            gamma[(long)k * nsel + i] = fpA * fpB + fxA * fxB;
            tau[(long)k * nsel + i] = (ox * dxt[0] + oy * dxt[1] + oz * dxt[2]) / ORC_C_LIGHT;
        }
    }
    free(xyz);
    return 0;
}

int orc_geometry(const double det[6], int nside, int nt, double t0, double stride, double dur,
                 double *gamma, double *tau)
{
    return orc_geometry_at(det, nside, nt, t0, stride, dur, 12L * nside * nside, NULL, gamma, tau);
}

/* ------------------------------------------------------------------------ */
/* One dirty-map / Fisher-diagonal element, straight from the definition.     */
/* C is interleaved complex [nt][ld] (re, im), w is [nt][ld]; column c of the  */
/* call holds absolute bin k0 + c with frequency f0 + (k0 + c) * df.           */
/* Also returns S = sum_t |w gamma| |C|, the scale used for the error of X.    */
/* ------------------------------------------------------------------------ */
static void one_term(int nt, long ld, long npix, const double *C, const double *w, double f,
                     long col, const double *gamma, const double *tau, long p,
                     double *X, double *G, double *S)
{
    double x = 0.0, g = 0.0, s = 0.0;
    for (int t = 0; t < nt; ++t) {
        double cr = C[2 * ((long)t * ld + col)], ci = C[2 * ((long)t * ld + col) + 1];
        double wt = w[(long)t * ld + col];
        double gm = gamma[(long)t * npix + p];
        double ph = 2.0 * ORC_PI * f * tau[(long)t * npix + p];
        x += wt * gm * (cr * cos(ph) - ci * sin(ph));
        g += wt * gm * gm;
        s += fabs(wt * gm) * sqrt(cr * cr + ci * ci);
    }
    *X = x;
    *G = g;
    if (S) *S = s;
}

/* Full maps X[nf][npix], G[nf][npix] (and optionally S).  OpenMP over pixels. */
void orc_maps(int nt, int nf, long ld, long npix, const double *C, const double *w, double f0,
              double df, long k0, const double *gamma, const double *tau, double *X, double *G,
              double *S, int nthreads)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (long p = 0; p < npix; ++p) {
        for (int c = 0; c < nf; ++c) {
            double f = f0 + (double)(k0 + c) * df;
            one_term(nt, ld, npix, C, w, f, c, gamma, tau, p, &X[(long)c * npix + p],
                     &G[(long)c * npix + p], S ? &S[(long)c * npix + p] : NULL);
        }
    }
}

/* Selected (column, pixel) elements only. */
void orc_maps_at(int nt, long ld, long npix, const double *C, const double *w, double f0, double df,
                 long k0, const double *gamma, const double *tau, long nsel, const int64_t *cols,
                 const int64_t *pix, double *X, double *G, double *S, int nthreads)
{
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads > 0 ? nthreads : 1)
    for (long i = 0; i < nsel; ++i) {
        double f = f0 + (double)(k0 + cols[i]) * df;
        one_term(nt, ld, npix, C, w, f, cols[i], gamma, tau, pix[i], &X[i], &G[i], S ? &S[i] : NULL);
    }
}

/* Broadband sums over columns [klo, khi) (Sec. V).  H is indexed by column. */
void orc_band(int nf, long npix, const double *X, const double *G, const double *H, int klo,
              int khi, double *Xbb, double *Gbb)
{
    (void)nf;
    for (long p = 0; p < npix; ++p) {
        double xs = 0.0, gs = 0.0;
        for (int k = klo; k < khi; ++k) {
            xs += X[(long)k * npix + p];
            gs += H[k] * G[(long)k * npix + p];
        }
        Xbb[p] = xs;
        Gbb[p] = gs;
    }
}

/* ------------------------------------------------------------------------ */
/* Fisher diagonal with the overlapping-window neighbour terms (Sec. II.B,    */
/* Eq. fwGamma with p = p'), straight from the definition:                    */
/*   G(k,p) = sum_t conj(K_t) [ K_t v_t - K_{t-1} u_t - K_{t+1} w_t ],         */
/*   K_t = gamma(t,p) exp(+2 pi i f_k tau(t,p)).                              */
/* The folded day is periodic (the geometry repeats every sidereal day):      */
/* segment 0's predecessor is segment nt - 1 and segment nt - 1's successor   */
/* is segment 0.  Returns the real part G, the imaginary part Gi (zero when    */
/* u_t = w_{t-1}, as the folded series are) and the scale                     */
/*   S = sum_t |v_t| g_t^2 + |u_t| |g_t g_{t-1}| + |w_t| |g_t g_{t+1}|.        */
/* v, u, w are [nt][ld]; column c is absolute bin k0 + c.                      */
/* ------------------------------------------------------------------------ */
static void overlap_term(int nt, long ld, long npix, const double *v, const double *u,
                         const double *wn, double f, long col, const double *gamma,
                         const double *tau, long p, double *G, double *Gi, double *S)
{
    double gr = 0.0, gi = 0.0, s = 0.0;
    for (int t = 0; t < nt; ++t) {
        const double gt = gamma[(long)t * npix + p];
        const double pt = 2.0 * ORC_PI * f * tau[(long)t * npix + p];
        const double kr = gt * cos(pt), ki = gt * sin(pt); /* K_t */
        /* bracket B = K_t v_t - K_{t-1} u_t - K_{t+1} w_t */
        const double vt = v[(long)t * ld + col];
        double br = kr * vt, bi = ki * vt;
        s += fabs(vt) * gt * gt;
        {
            const int tp = t >= 1 ? t - 1 : nt - 1; /* predecessor, periodic */
            const double g1 = gamma[(long)tp * npix + p];
            const double p1 = 2.0 * ORC_PI * f * tau[(long)tp * npix + p];
            const double ut = u[(long)t * ld + col];
            br -= g1 * cos(p1) * ut;
            bi -= g1 * sin(p1) * ut;
            s += fabs(ut) * fabs(gt * g1);
        }
        {
            const int tn = t + 1 < nt ? t + 1 : 0; /* successor, periodic */
            const double g1 = gamma[(long)tn * npix + p];
            const double p1 = 2.0 * ORC_PI * f * tau[(long)tn * npix + p];
            const double wt = wn[(long)t * ld + col];
            br -= g1 * cos(p1) * wt;
            bi -= g1 * sin(p1) * wt;
            s += fabs(wt) * fabs(gt * g1);
        }
        /* conj(K_t) * B */
        gr += kr * br + ki * bi;
        gi += kr * bi - ki * br;
    }
    *G = gr;
    if (Gi) *Gi = gi;
    if (S) *S = s;
}

/* Selected (column, pixel) elements of the overlap-corrected Fisher diagonal. */
void orc_fisher_overlap_at(int nt, long ld, long npix, const double *v, const double *u,
                           const double *wn, double f0, double df, long k0, const double *gamma,
                           const double *tau, long nsel, const int64_t *cols, const int64_t *pix,
                           double *G, double *Gi, double *S, int nthreads)
{
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads > 0 ? nthreads : 1)
    for (long i = 0; i < nsel; ++i) {
        double f = f0 + (double)(k0 + cols[i]) * df;
        overlap_term(nt, ld, npix, v, u, wn, f, cols[i], gamma, tau, pix[i], &G[i], Gi ? &Gi[i] : NULL,
                     S ? &S[i] : NULL);
    }
}

/* ------------------------------------------------------------------------ */
/* Folding (Sec. II.B): ndays days of nt segments, absolute segment a = d nt + */
/* tau.  Per present segment a and bin, with eps = W when the neighbour a +- 1 */
/* exists and is present (0 otherwise):                                       */
/*   v_tau += s_a                                                             */
/*   u_tau += eps_{a-1} (s_a + s_{a-1}) / 2,  w_tau += eps_{a+1} (s_a + s_{a+1}) / 2 */
/*   x_tau += s_a C_a - eps_{a-1} (s_a + s_{a-1}) / 2 C_{a-1}                  */
/*                    - eps_{a+1} (s_a + s_{a+1}) / 2 C_{a+1}                  */
/* C interleaved complex [ndays][nt][ld], s [ndays][nt][ld], present           */
/* [ndays][nt] (nonzero = data); outputs v, u, w [nt][nf], x complex [nt][nf].  */
/* ------------------------------------------------------------------------ */
void orc_fold(int ndays, int nt, int nf, long ld, const double *C, const double *sv,
              const unsigned char *present, double W, double *v, double *u, double *w, double *x)
{
    const long nseg = (long)ndays * nt;
    for (int tau = 0; tau < nt; ++tau)
        for (int c = 0; c < nf; ++c) {
            double vs = 0.0, us = 0.0, ws = 0.0, xr = 0.0, xi = 0.0;
            for (int d = 0; d < ndays; ++d) {
                const long a = (long)d * nt + tau;
                if (!present[a]) continue;
                const double sa = sv[a * ld + c];
                vs += sa;
                xr += sa * C[2 * (a * ld + c)];
                xi += sa * C[2 * (a * ld + c) + 1];
                if (a - 1 >= 0 && present[a - 1]) {
                    const double e = 0.5 * W * (sa + sv[(a - 1) * ld + c]);
                    us += e;
                    xr -= e * C[2 * ((a - 1) * ld + c)];
                    xi -= e * C[2 * ((a - 1) * ld + c) + 1];
                }
                if (a + 1 < nseg && present[a + 1]) {
                    const double e = 0.5 * W * (sa + sv[(a + 1) * ld + c]);
                    ws += e;
                    xr -= e * C[2 * ((a + 1) * ld + c)];
                    xi -= e * C[2 * ((a + 1) * ld + c) + 1];
                }
            }
            v[(long)tau * nf + c] = vs;
            u[(long)tau * nf + c] = us;
            w[(long)tau * nf + c] = ws;
            x[2 * ((long)tau * nf + c)] = xr;
            x[2 * ((long)tau * nf + c) + 1] = xi;
        }
}

/* ------------------------------------------------------------------------ */
/* Network sum over baselines (the sum over I of Eq. eq:narrowband): the      */
/* element-wise sum of nmaps maps of n values, in map order.                  */
/* ------------------------------------------------------------------------ */
void orc_network_sum(int nmaps, long n, const double *maps, double *out)
{
    for (long i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int m = 0; m < nmaps; ++m) acc += maps[(long)m * n + i];
        out[i] = acc;
    }
}

/* ------------------------------------------------------------------------ */
/* Directed and isotropic contractions (Sec. V): per row k of a map M[nf][npix] */
/* the sum over the pixels of a set (the pixels that contain a source), or     */
/* over all pixels when nsel < 0; HEALPix pixels have equal area, so no        */
/* weights.                                                                   */
/* ------------------------------------------------------------------------ */
void orc_contract(int nf, long npix, const double *M, int nsel, const int64_t *pix, double *out)
{
    for (int k = 0; k < nf; ++k) {
        double acc = 0.0;
        if (nsel < 0)
            for (long p = 0; p < npix; ++p) acc += M[(long)k * npix + p];
        else
            for (int j = 0; j < nsel; ++j) acc += M[(long)k * npix + pix[j]];
        out[k] = acc;
    }
}

/* ------------------------------------------------------------------------ */
/* Full Fisher information matrix of a band (Eq. eq_fisher; the broadband     */
/* spectral weighting of Sec. V as for the diagonal):                         */
/*   G(p,p') = sum_{c in [clo,chi)} H_c sum_t w(t,c) Re[conj(K_p) K_p'],        */
/*   K_p = gamma(t,p) exp(+2 pi i f_c tau(t,p))                                 */
/*         => gamma_p gamma_p' cos 2 pi f_c (tau_p - tau_p').                  */
/* w is [nt][ld] (column c = bin k0 + c), H is indexed by column; G[npix][npix]. */
/* OpenMP over rows.                                                          */
/* ------------------------------------------------------------------------ */
void orc_fisher_full(int nt, long ld, long npix, const double *w, const double *H, double f0, double df,
                     long k0, int clo, int chi, const double *gamma, const double *tau, double *G,
                     int nthreads)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (long p = 0; p < npix; ++p)
        for (long q = 0; q < npix; ++q) {
            double acc = 0.0;
            for (int c = clo; c < chi; ++c) {
                const double f = f0 + (double)(k0 + c) * df;
                double s = 0.0;
                for (int t = 0; t < nt; ++t) {
                    const double gp = gamma[(long)t * npix + p], gq = gamma[(long)t * npix + q];
                    const double d = tau[(long)t * npix + p] - tau[(long)t * npix + q];
                    s += w[(long)t * ld + c] * gp * gq * cos(2.0 * ORC_PI * f * d);
                }
                acc += H[c] * s;
            }
            G[p * npix + q] = acc;
        }
}

// Host FP64 solve of the JTFS plan (validation, filterbank centres and widths,
// critical-rate schedule, padded shapes, workspace layout).  No GPU calls.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace jtfs {

static thread_local std::string g_err;
void set_error(const std::string& s) { g_err = s; }
const char* last_error() { return g_err.c_str(); }

static bool pow2(int64_t v) { return v >= 1 && (v & (v - 1)) == 0; }
static int ilog2(int64_t v) { int k = 0; while ((int64_t(1) << k) < v) ++k; return k; }
static int64_t rup(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// xi / sigma of a Gaussian-spectrum wavelet whose neighbours 2^(1/Q) apart cross
// at -3 dB; one wavelet per octave gives about 2.5 (sec. 3.3).
static double quality_factor(int Q) {
    const double rho = std::pow(2.0, -1.0 / Q);
    return (1.0 + rho) / (1.0 - rho) * std::sqrt(std::log(2.0));
}

// Largest k in [0, cap] leaving a decimated Nyquist 2^-(k+1) of at least kCEnv*sigma
// (sec. 1: the critical sample rate depends on the band).
static int critical_log2(double sigma, int cap) {
    const double v = 1.0 / (2.0 * kCEnv * sigma);
    int k = v >= 1.0 ? (int)std::floor(std::log2(v)) : 0;
    return std::min(std::max(k, 0), cap);
}

// Centres and widths of a Morlet family: constant-Q wavelets xi_max 2^(-n/Q) down
// to the minimum width kSigma0/2^Jp, then minimum-width wavelets spaced by their
// -3 dB width (eq. 1 dilations, discretised).
static bool family_centres(int Jp, int Q, std::vector<double>* xi, std::vector<double>* sg) {
    const double Qf = quality_factor(Q);
    const double xi_max = std::max(1.0 / (1.0 + std::pow(2.0, 1.0 / Q)), 0.35);
    const double smin = kSigma0 / std::pow(2.0, Jp);
    xi->clear(); sg->clear();
    for (int n = 0;; ++n) {
        const double c = xi_max * std::pow(2.0, -(double)n / Q);
        if (c / Qf < smin) break;
        xi->push_back(c);
        sg->push_back(c / Qf);
        if (n > 100000) return false;
    }
    if (xi->empty()) return false;
    const double delta = 2.0 * std::sqrt(std::log(2.0)) * smin;
    const double xc = xi->back();
    for (int k = 1; xc - k * delta >= delta; ++k) {
        xi->push_back(xc - k * delta);
        sg->push_back(smin);
    }
    return true;
}

// Bins of an M-point grid (f = m/M, 0 <= m <= M/2) where the un-normalised
// Morlet spectrum can exceed kSupportTol / 2.
static void family_supports(Family* f) {
    const int n = f->n();
    f->lo.resize(n); f->hi.resize(n); f->off.resize(n);
    const double R = std::sqrt(2.0 * std::log(2.0 / kSupportTol));
    int64_t off = 0;
    for (int i = 0; i < n; ++i) {
        double a = (f->xi[i] - R * f->sigma[i]) * f->M, b = (f->xi[i] + R * f->sigma[i]) * f->M;
        int lo = (int)std::max(0.0, std::floor(a));
        int hi = (int)std::min((double)(f->M / 2), std::ceil(b));
        if (lo > hi) lo = hi;
        f->lo[i] = lo; f->hi[i] = hi; f->off[i] = off;
        off += hi - lo + 1;
    }
    f->total = off;
}

int solve_shapes(const jtfs_params& p, Shapes* s) {
    *s = Shapes{};
    s->p = p;
    if (!pow2(p.N) || !pow2(p.T) || !pow2(p.F)) { set_error("N, T and F must be powers of two"); return JTFS_EINVAL; }
    if (p.N < 16 || p.N > (int64_t(1) << 24)) { set_error("N must lie in [2^4, 2^24]"); return JTFS_EINVAL; }
    if (p.T > p.N) { set_error("T must not exceed N"); return JTFS_EINVAL; }
    if (p.flags & ~(JTFS_NO_FREQ_AVERAGE | JTFS_TIME_SCATTERING | JTFS_LOWPASS_PAIRS | JTFS_UNPAD_LAMBDA)) {
        set_error("unknown flag bits"); return JTFS_EINVAL; }
    if ((p.flags & JTFS_NO_FREQ_AVERAGE) && (p.flags & JTFS_TIME_SCATTERING)) {
        set_error("JTFS_NO_FREQ_AVERAGE and JTFS_TIME_SCATTERING exclude each other"); return JTFS_EINVAL; }
    if ((p.flags & JTFS_TIME_SCATTERING) && (p.flags & (JTFS_LOWPASS_PAIRS | JTFS_UNPAD_LAMBDA))) {
        set_error("JTFS_LOWPASS_PAIRS and JTFS_UNPAD_LAMBDA need the frequential stage (not JTFS_TIME_SCATTERING)");
        return JTFS_EINVAL; }
    if ((p.flags & JTFS_NO_FREQ_AVERAGE) && (p.flags & JTFS_UNPAD_LAMBDA)) {
        set_error("JTFS_UNPAD_LAMBDA applies to the frequency-averaged output (not JTFS_NO_FREQ_AVERAGE)");
        return JTFS_EINVAL; }
    s->avg_fr = !(p.flags & JTFS_NO_FREQ_AVERAGE);
    s->tscat = (p.flags & JTFS_TIME_SCATTERING) != 0;
    s->complete = (p.flags & JTFS_LOWPASS_PAIRS) != 0;
    if (p.Q1 < 1 || p.Q2 < 1 || p.Q_fr < 1 || p.Q1 > 64 || p.Q2 > 64 || p.Q_fr > 64) {
        set_error("Q1, Q2 and Q_fr must lie in [1, 64]"); return JTFS_EINVAL; }
    s->N = p.N; s->T = p.T; s->F = p.F;
    s->logN = ilog2(p.N); s->logT = ilog2(p.T); s->logF = ilog2(p.F);
    if (p.J < 1 || p.J > s->logN) { set_error("J must lie in [1, log2 N]"); return JTFS_EINVAL; }

    // first order, cycles/sample on the N grid
    Family& f1 = s->f1;
    f1.M = (int)p.N;
    if (!family_centres(p.J, p.Q1, &f1.xi, &f1.sigma)) { set_error("first-order filterbank is empty"); return JTFS_EINVAL; }
    s->n1 = f1.n();
    s->kX = std::min(s->logT, critical_log2(f1.sigma[0], s->logN));
    s->NX = p.N >> s->kX;
    s->logNX = s->logN - s->kX;
    if (p.J - s->kX < 1) { set_error("J - kX must be >= 1"); return JTFS_EINVAL; }

    // second order, cycles per scalogram sample on the NX grid
    Family& f2 = s->f2;
    f2.M = (int)s->NX;
    if (!family_centres(p.J - s->kX, p.Q2, &f2.xi, &f2.sigma)) { set_error("second-order filterbank is empty"); return JTFS_EINVAL; }
    s->n_alpha_psi = f2.n();
    s->n_alpha = f2.n() + (s->complete ? 1 : 0);     // the last rate: the lowpass phi_T

    // frequential, cycles per lambda bin on the zero-padded L grid
    s->logL = ilog2(s->n1);
    s->L = 1 << s->logL;
    if (p.J_fr < 1 || p.J_fr > s->logL) { set_error("J_fr must lie in [1, log2 L]"); return JTFS_EINVAL; }
    if (p.F > s->L) { set_error("F must not exceed L"); return JTFS_EINVAL; }
    Family& ff = s->ffr;
    ff.M = s->L;
    if (!family_centres(p.J_fr, p.Q_fr, &ff.xi, &ff.sigma)) { set_error("frequential filterbank is empty"); return JTFS_EINVAL; }
    s->n_beta_psi = ff.n();
    s->n_beta = ff.n() + (s->complete ? 1 : 0);       // the last scale: the lowpass phi_F

    family_supports(&f1);
    family_supports(&f2);
    family_supports(&ff);

    // schedules and padded shapes
    s->NT = (int)(p.N / p.T);
    s->NTp = (int)rup(s->NT, 32);
    s->NL = (int)(s->L / p.F);
    // unpadded: the rows m whose log-frequency m F falls on a first-order band (m F < n1)
    s->NLo = (p.flags & JTFS_UNPAD_LAMBDA) ? (int)((s->n1 + p.F - 1) / p.F) : s->NL;
    s->Kp = (int)rup(s->n1, kKStep);
    s->k2.resize(s->n_alpha); s->Ta.resize(s->n_alpha); s->Tp.resize(s->n_alpha);
    s->yoff.resize(s->n_alpha); s->phioff.resize(s->n_alpha);
    int64_t yo = 0, po = 0;
    for (int a = 0; a < s->n_alpha; ++a) {
        // phi_T keeps the capped rate: its rows land on the N/T frames undecimated
        s->k2[a] = a < s->n_alpha_psi ? critical_log2(f2.sigma[a], s->logT - s->kX) : s->logT - s->kX;
        s->Ta[a] = (int)(s->NX >> s->k2[a]);
        s->Tp[a] = std::max(s->Ta[a], kTileTh);
        s->yoff[a] = yo; s->phioff[a] = po;
        yo += (int64_t)s->Kp * s->Tp[a];
        po += (int64_t)s->Tp[a] * s->NTp;
        s->sumT += s->Ta[a];
    }
    s->sumTp = yo / s->Kp;
    set_chunks(s, kChunkT);
    s->kfr.resize(s->n_beta); s->Lb.resize(s->n_beta); s->rowoff.resize(s->n_beta); s->pfoff.resize(s->n_beta);
    int ro = 0; int64_t pf = 0;
    for (int b = 0; b < s->n_beta; ++b) {
        s->kfr[b] = critical_log2(b < s->n_beta_psi ? ff.sigma[b] : kSigma0 / (double)p.F, s->logF);
        s->Lb[b] = s->L >> s->kfr[b];
        s->rowoff[b] = ro; ro += s->Lb[b];
        s->pfoff[b] = pf; pf += (int64_t)s->NL * s->Lb[b];
    }
    s->Mh = ro;
    s->Mp = (int)rup(ro, kTileL);
    // phi_T support on the NX grid (frequency m/N cycles/sample)
    {
        const double sg = kSigma0 / (double)p.T;
        const double mm = (double)p.N * sg * std::sqrt(2.0 * std::log(1.0 / kSupportTol));
        s->Mphi = (int)std::min<double>((double)(s->NX / 2), std::floor(mm) + 1.0);
    }
    return JTFS_OK;
}

void set_chunks(Shapes* s, int chunk) {
    s->chunk.resize(s->n_alpha); s->nch.resize(s->n_alpha); s->vchoff.resize(s->n_alpha);
    int64_t co = 0;
    for (int a = 0; a < s->n_alpha; ++a) {
        s->chunk[a] = std::min(s->Tp[a], chunk);
        s->nch[a] = s->Tp[a] / s->chunk[a];
        s->vchoff[a] = co;
        co += s->nch[a];
    }
    s->sumch = co;
}

int check_supported(const Shapes& s) {
    if (s.logNX > kMaxLogNX) {
        set_error("scalogram length N/2^kX above 2^15 is not supported by this library");
        return JTFS_ENOTSUP;
    }
    return JTFS_OK;
}

Workspace layout(const Shapes& s, int64_t B, bool with_split, bool with_pq, bool with_phase) {
    Workspace w;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += (bytes + 255) / 256 * 256; return r; };
    w.xh_pitch = s.N / 2 + 1;
    w.Xh_pitch = s.NX / 2 + 1;
    w.xh = take(sizeof(float2) * B * w.xh_pitch);
    w.tmp = take(sizeof(float2) * B * (s.N / 2));
    w.tmp64 = take(sizeof(double2) * B * (s.N / 2));     // input transform in FP64
    w.z64 = take(sizeof(double2) * B * (s.N / 2));
    w.Xh = take(sizeof(float2) * B * s.n1 * w.Xh_pitch);
    w.Y2 = take(sizeof(float2) * B * s.Kp * s.sumTp);
    w.Yh = take(with_split ? sizeof(float2) * B * s.Kp * s.sumTp : 0);   // 4 halves per complex value
    w.rowmax = take(sizeof(float) * B * s.n_alpha * s.Kp);
    w.yscale = take(sizeof(float) * B * s.n_alpha);
    // partial V: per signal, per (alpha, t-chunk, t-half) slot, per l-tile, spin, tau, l
    w.vp_bstride = s.sumch * 2 * (s.Mp / kTileL) * 2 * (int64_t)s.NTp * kTileL;
    w.Vp = take(sizeof(float) * B * w.vp_bstride);
    w.ph_bstride = (int64_t)2 * s.sumTp * s.Mp;
    w.phase = take(with_phase ? sizeof(uint32_t) * B * w.ph_bstride : 0);
    w.fwd_total = o;                 // the forward touches nothing beyond this point
    w.gvmax = take(sizeof(float) * B * s.n_alpha * 2 * s.n_beta);
    w.gV = take(sizeof(float) * B * s.n_alpha * 2 * s.Mp * s.NTp);
    int64_t maxTp = 0;
    for (int a = 0; a < s.n_alpha; ++a) maxTp = std::max<int64_t>(maxTp, s.Tp[a]);
    w.PQ = take(with_pq ? sizeof(float2) * B * 2 * s.Mp * maxTp : 0);
    w.gY2 = take(sizeof(float2) * B * s.Kp * s.sumTp);
    w.gX = take(sizeof(float) * B * s.n1 * s.NX);
    w.g1 = take(sizeof(float2) * B * s.n1 * s.NX);
    w.gxh = take(sizeof(float2) * B * w.xh_pitch);
    // gV split for the backward from the stored phase: per rate and 32-row chunk, the
    // FP16 planes of both spins and the rows' scales
    w.gvs_bstride = (int64_t)s.n_alpha * (s.Mp / 32) * (512 * (s.NTp / 32) + 16);
    w.gvs = take(with_phase ? 16 * B * w.gvs_bstride : 0);
    w.total = o;
    return w;
}

}  // namespace jtfs

extern "C" {

const char* jtfs_last_error(void) { return jtfs::last_error(); }

int jtfs_query(const jtfs_params* p, jtfs_info* out) {
    if (!p || !out) { jtfs::set_error("null pointer"); return JTFS_EINVAL; }
    jtfs::Shapes s;
    int st = jtfs::solve_shapes(*p, &s);
    if (st != JTFS_OK) return st;
    std::memset(out, 0, sizeof(*out));
    out->n1 = s.n1; out->n_alpha = s.n_alpha; out->n_beta = s.n_beta; out->L = s.L; out->kX = s.kX;
    out->M_h = s.Mh; out->NX = s.NX; out->out_t = s.NT; out->out_l = s.NLo; out->sum_T = s.sumT;
    out->s1_per_signal = (int64_t)s.n1 * s.NT;
    out->s2_per_signal = s.tscat    ? (int64_t)s.n_alpha * s.n1 * s.NT
                         : s.avg_fr ? (int64_t)s.n_alpha * s.n_beta * 2 * s.NLo * s.NT
                                    : (int64_t)s.n_alpha * 2 * s.Mh * s.NT;
    const jtfs::Workspace w = jtfs::layout(s, 1, true, true, false);
    out->ws_fwd = (int64_t)w.fwd_total;
    out->ws_bwd = (int64_t)w.total;
    return st;
}

int jtfs_query_filters(const jtfs_params* p, int family, int32_t cap, double* xi, double* sigma,
                       int32_t* log2_decim, int32_t* count) {
    if (!p || !count) { jtfs::set_error("null pointer"); return JTFS_EINVAL; }
    jtfs::Shapes s;
    int st = jtfs::solve_shapes(*p, &s);
    if (st != JTFS_OK) return st;
    const jtfs::Family* f = family == 0 ? &s.f1 : family == 1 ? &s.f2 : family == 2 ? &s.ffr : nullptr;
    if (!f) { jtfs::set_error("family must be 0, 1 or 2"); return JTFS_EINVAL; }
    *count = f->n();
    if (f->n() > cap) { jtfs::set_error("cap too small"); return JTFS_EINVAL; }
    for (int i = 0; i < f->n(); ++i) {
        if (xi) xi[i] = f->xi[i];
        if (sigma) sigma[i] = f->sigma[i];
        if (log2_decim) log2_decim[i] = family == 0 ? s.kX : family == 1 ? s.k2[i] : s.kfr[i];
    }
    return JTFS_OK;
}

}  // extern "C"

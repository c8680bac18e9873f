/* Test infrastructure (oracle): the reactor right-hand side, written once over
 * a scalar type and included twice by oracle.c -- for SC = double and for
 * SC = double complex (complex-step derivatives).  Nothing here clips, takes
 * an absolute value or branches on the state, so the complex version stays
 * analytic.
 *
 * What is computed is the plain definition of an adiabatic, constant-pressure,
 * ideal-gas homogeneous reactor: the paper models every CFD cell as an
 * independent homogeneous gas-phase reactor (Sec. 1) whose species source
 * terms feed the species and enthalpy transport equations (Sec. 2.1, Eqs. 3-4).
 * The paper prints no rate laws; the textbook CHEMKIN conventions are used:
 *   k    = exp(dlnA) * A * T^b * exp(-Ea/(R T))
 *   [M]  = sum_k alpha_k C_k                  (third-body and fall-off)
 *   Troe: Pr = k0[M]/kinf, Fcent = (1-a)e^{-T/T3} + a e^{-T/T1} + e^{-T2/T},
 *         c = -0.4-0.67 log Fcent, n = 0.75-1.27 log Fcent,
 *         f = (log Pr + c)/(n - 0.14 (log Pr + c)), log F = log Fcent/(1+f^2),
 *         kf = kinf Pr/(1+Pr) F                 (base-10 logarithms)
 *   ln Kc = -sum_k nu_k g_k/RT + (sum_k nu_k) ln(p0/(R T)),  kr = kf/Kc
 *   q    = kf prod C^nu' - kr prod C^nu''   (times [M] for third-body)
 *   dY_k/dt = W_k wdot_k / rho,  dT/dt = -sum_k h_k wdot_k / (rho cp)
 * with rho = p Wbar/(R T), C_k = rho Y_k/W_k.
 * The constant-volume variant (adiabatic, rigid vessel) holds rho fixed
 * instead of p (the argument p then carries rho), so C_k = rho Y_k/W_k with
 * that rho, and the energy balance is on internal energy:
 *   dT/dt = -sum_k u_k wdot_k / (rho cv),  u_k = h_k - R T,  cv = cp - R/Wbar.
 *
 * Expects: SC, FN(name) (function-name decoration), SEXP, SLOG, SPOW.
 */

/* NASA-7 single-range thermodynamics of species k at temperature T. */
static void FN(thermo)(const omech *m, int k, SC T, SC *cp_R, SC *h_RT, SC *s_R)
{
    const double *a = m->nasa + 7 * k;
    SC T2 = T * T, T3 = T2 * T, T4 = T3 * T;
    *cp_R = a[0] + a[1] * T + a[2] * T2 + a[3] * T3 + a[4] * T4;
    *h_RT = a[0] + a[1] * T / 2.0 + a[2] * T2 / 3.0 + a[3] * T3 / 4.0 + a[4] * T4 / 5.0 + a[5] / T;
    *s_R = a[0] * SLOG(T) + a[1] * T + a[2] * T2 / 2.0 + a[3] * T3 / 3.0 + a[4] * T4 / 4.0 + a[6];
}

/* Rates of progress and production rates.  y = (Y_0..Y_{N-1}, T); p is the
 * pressure, or with constv != 0 the density rho;
 * dlnA[j] (may be NULL) multiplies reaction j's net rate by exp(dlnA[j]).
 * Outputs (any may be NULL): kf[R], kr[R], q[R], wdot[N] (mol/m^3/s),
 * and through aux[4]: rho, cp (J/kg/K), sum_k h_k wdot_k, Wbar. */
static void FN(rates)(const omech *m, double p, const SC *y, const SC *dlnA, SC *kf_out,
                      SC *kr_out, SC *q_out, SC *wdot, SC *aux, int constv)
{
    const int N = m->N;
    const double R = m->R;
    SC T = y[N];
    SC cpR[OM_MAXSP], hRT[OM_MAXSP], sR[OM_MAXSP], C[OM_MAXSP];
    SC sumYW = 0.0;
    for (int k = 0; k < N; ++k) {
        FN(thermo)(m, k, T, &cpR[k], &hRT[k], &sR[k]);
        sumYW += y[k] / m->W[k];
    }
    SC Wbar = 1.0 / sumYW;
    SC rho = constv ? (SC)p : p * Wbar / (R * T);
    SC cp = 0.0;
    for (int k = 0; k < N; ++k) {
        C[k] = rho * y[k] / m->W[k];
        cp += R * cpR[k] * y[k] / m->W[k];
    }
    if (wdot)
        for (int k = 0; k < N; ++k) wdot[k] = 0.0;
    SC lnT = SLOG(T);
    for (int j = 0; j < m->R_; ++j) {
        const omrxn *r = &m->rx[j];
        SC dl = dlnA ? dlnA[j] : (SC)0.0;
        int order = 0;
        for (int i = 0; i < r->nr; ++i) order += r->nu_r[i];
        SC M = 0.0;
        if (r->kind != RX_PLAIN) {
            for (int k = 0; k < N; ++k) M += r->alpha[k] * C[k];
        }
        /* A in cgs -> SI: (cm^3/mol)^(m-1)/s -> (m^3/mol)^(m-1)/s */
        int m_inf = order + (r->kind == RX_THIRD ? 1 : 0);
        double Ainf = pow(10.0, r->log10A) * pow(10.0, -6.0 * (m_inf - 1));
        SC kinf = SEXP(dl) * Ainf * SEXP(r->b * lnT) * SEXP(-r->Ea / (R * T));
        SC kf;
        if (r->kind == RX_TROE) {
            double A0 = pow(10.0, r->troe[0]) * pow(10.0, -6.0 * order);
            SC k0 = SEXP(dl) * A0 * SEXP(r->troe[1] * lnT) * SEXP(-r->troe[2] / (R * T));
            double a = r->troe[3], T3 = r->troe[4], T1 = r->troe[5], T2 = r->troe[6];
            SC Pr = k0 * M / kinf;
            SC Fcent = (1.0 - a) * SEXP(-T / T3) + a * SEXP(-T / T1) + SEXP(-T2 / T);
            SC lFc = SLOG(Fcent) / M_LN10;
            SC cc = -0.4 - 0.67 * lFc;
            SC nn = 0.75 - 1.27 * lFc;
            SC x = SLOG(Pr) / M_LN10 + cc;
            SC f1 = x / (nn - 0.14 * x);
            SC lF = lFc / (1.0 + f1 * f1);
            kf = kinf * (Pr / (1.0 + Pr)) * SPOW(10.0, lF);
        } else {
            kf = kinf;
        }
        SC dgsum = 0.0;
        int dnu = 0;
        for (int i = 0; i < r->nr; ++i) {
            dgsum -= (SC)r->nu_r[i] * (hRT[r->sp_r[i]] - sR[r->sp_r[i]]);
            dnu -= r->nu_r[i];
        }
        for (int i = 0; i < r->np; ++i) {
            dgsum += (SC)r->nu_p[i] * (hRT[r->sp_p[i]] - sR[r->sp_p[i]]);
            dnu += r->nu_p[i];
        }
        SC lnKc = -dgsum + (double)dnu * SLOG(m->p0 / (R * T));
        SC kr = kf * SEXP(-lnKc);
        SC pf = 1.0, pr = 1.0;
        for (int i = 0; i < r->nr; ++i)
            for (int v = 0; v < r->nu_r[i]; ++v) pf *= C[r->sp_r[i]];
        for (int i = 0; i < r->np; ++i)
            for (int v = 0; v < r->nu_p[i]; ++v) pr *= C[r->sp_p[i]];
        SC q = kf * pf - kr * pr;
        if (r->kind == RX_THIRD) q *= M;
        if (kf_out) kf_out[j] = kf;
        if (kr_out) kr_out[j] = kr;
        if (q_out) q_out[j] = q;
        if (wdot) {
            for (int i = 0; i < r->nr; ++i) wdot[r->sp_r[i]] -= (double)r->nu_r[i] * q;
            for (int i = 0; i < r->np; ++i) wdot[r->sp_p[i]] += (double)r->nu_p[i] * q;
        }
    }
    if (aux) {
        SC hw = 0.0;
        if (wdot)
            for (int k = 0; k < N; ++k) hw += hRT[k] * R * T * wdot[k];
        aux[0] = rho;
        aux[1] = cp;
        aux[2] = hw;
        aux[3] = Wbar;
    }
}

/* f(y): dY_k/dt for k < N and dT/dt in f[N].  mode bits: OM_ISOTHERMAL
 * (f[N] = 0), OM_CONSTV (constant-volume reactor; p carries the density). */
static void FN(rhs)(const omech *m, double p, const SC *y, const SC *dlnA, SC *f, int mode)
{
    const int N = m->N;
    const int constv = (mode & OM_CONSTV) != 0;
    SC wdot[OM_MAXSP], aux[4];
    FN(rates)(m, p, y, dlnA, NULL, NULL, NULL, wdot, aux, constv);
    SC rho = aux[0], cp = aux[1], hw = aux[2], Wbar = aux[3];
    for (int k = 0; k < N; ++k) f[k] = m->W[k] * wdot[k] / rho;
    if (mode & OM_ISOTHERMAL) {
        f[N] = 0.0;
    } else if (constv) {
        SC sw = 0.0;
        for (int k = 0; k < N; ++k) sw += wdot[k];
        SC uw = hw - m->R * y[N] * sw;       /* sum_k (h_k - R T) wdot_k */
        SC cv = cp - m->R / Wbar;
        f[N] = -uw / (rho * cv);
    } else {
        f[N] = -hw / (rho * cp);
    }
}

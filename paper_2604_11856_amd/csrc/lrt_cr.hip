// gfx950 kernel of the quasi-steady-state collisional-radiative populations
// (arXiv 2604.11856, Sec. 2.1 CR model): one wave per (cell, species)
// assembles the l x l system R n = b of the QSS balance with the ground-state
// closure in LDS, one lane per row, and solves it by LU with partial
// pivoting.  The states are an atom's table levels or a diatomic molecule's
// electronic states.  The
// matrix is small (l <= 64) and every system is independent, so the work is a
// batch of wave-sized dense solves, bound by VALU latency and LDS traffic, not
// a contraction for the matrix cores.  Everything is FP64.
#include <hip/hip_runtime.h>

#include <cmath>

#include "lrt_device.h"
#include "lrt_internal.h"

namespace lrt {

namespace {

constexpr double kAvogadro = 6.02214076e23;      // mol^-1
constexpr double kMe = 9.1093837015e-28;         // electron mass, g

// Sec. 2.1 rate formula: k = C T^n exp(-E_a / T), cm^3 mol^-1 s^-1.
__device__ __forceinline__ double arrhenius(const double *t, double T)
{
    return t[0] * pow(T, t[1]) * exp(-t[2] / T);
}

__device__ __forceinline__ double rate_temperature(double a, double Ttr, double Tv)
{
    return pow(Ttr, a) * pow(Tv, 1.0 - a);
}

// Rate coefficient of the collisional transition i -> j (i != j) of one
// excitation table: Arrhenius of the pair at Tf upwards; downwards the
// detailed-balance reverse of the upward rate, evaluated at Tb with the state
// partition functions Qb (at Tb).
__device__ __forceinline__ double k_exc(const double *tab, int L, int i, int j, double Tf, double Tb,
                                        const double *Qb)
{
    if (j > i) return arrhenius(tab + 3 * (i * L + j), Tf);
    return arrhenius(tab + 3 * (j * L + i), Tb) * Qb[j] / Qb[i];
}

// Sum over the wave of one value per lane, in a fixed order; every lane
// receives the sum.
__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Partition functions of electronic state e of a molecule, in one pass over
// its (v, J) terms spread over the lanes: out[0] at (Tv, Tr) and out[1 + k]
// at T[k] (vibration and rotation alike, k < nT), each
// g_e e^{-c2 T_e/Tv} sum_v e^{-c2 G_v/Tv} sum_J (2J+1) e^{-c2 F_v(J)/Tr},
// F = B J(J+1) - D J^2 (J+1)^2.  Called by the whole wave; every lane
// receives the values.
template <int nT>
__device__ void mol_state_q(const DevSpecies &sp, int64_t e, double Tv, double Tr, const double *T, int lane,
                            double *out)
{
    const int64_t v0 = sp.vib_off[e];
    const int nv = (int)(sp.vib_off[e + 1] - v0), nJ = sp.el_Jmax[e] + 1;
    double iT[nT];
#pragma unroll
    for (int k = 0; k < nT; ++k) iT[k] = 1.0 / T[k];
    const double iTv = 1.0 / Tv, iTr = 1.0 / Tr;
    double acc[nT + 1];
#pragma unroll
    for (int k = 0; k <= nT; ++k) acc[k] = 0.0;
    for (int t = lane; t < nv * nJ; t += 64) {
        const int64_t v = v0 + t / nJ;
        const double J = (double)(t % nJ), jj = J * (J + 1.0), g = 2.0 * J + 1.0;
        const double x = kC2 * sp.vib_G[v], y = kC2 * (sp.vib_B[v] * jj - sp.vib_D[v] * jj * jj);
        acc[0] += g * exp(-x * iTv - y * iTr);
#pragma unroll
        for (int k = 0; k < nT; ++k) acc[1 + k] += g * exp(-(x + y) * iT[k]);
    }
    const double cT = kC2 * sp.el_T[e], ge = sp.el_g[e];
    out[0] = ge * exp(-cT * iTv) * wave_sum(acc[0]);
#pragma unroll
    for (int k = 0; k < nT; ++k) out[1 + k] = ge * exp(-cT * iT[k]) * wave_sum(acc[1 + k]);
}

// Partition function of a dissociation product at T: an atom's level sum,
// else the given constant.
__device__ __forceinline__ double product_q(const DevSpecies &sp, int64_t lev0, int32_t n_lev, double Qc,
                                            double T)
{
    if (n_lev == 0) return Qc;
    double q = 0.0;
    for (int32_t k = 0; k < n_lev; ++k) q += sp.lev_g[lev0 + k] * exp(-kC2 * sp.lev_E[lev0 + k] / T);
    return q;
}

// LDS row stride of the augmented matrix [R | b] (L + 1 columns): odd, so the
// lanes of a column walk hit distinct banks.
__host__ __device__ constexpr int row_stride(int L) { return (L + 1) | 1; }

__global__ __launch_bounds__(64) void cr_kernel(DevSpecies sp, DevCells cells, DevCR cr, const CellSpecies *cs)
{
    extern __shared__ double lds[];
    const int lane = threadIdx.x;
    const int r = blockIdx.x % cr.n;
    const int c = blockIdx.x / cr.n;
    const CRRec R = cr.rec[r];
    const int L = R.n_model, NL = R.n_lev, S = cells.n_species;
    const int ld = row_stride(L);
    const bool mol = R.kind == 2;
    double *M = lds;                 // [L][ld]: R, then b in column L
    double *QH = M + L * ld;         // [NL] state partition functions at the HPIE backward T
    double *QE = QH + NL;            // [NL] ... at the EIE backward T
    double *Qv = QE + NL;            // [NL] ... at (T_v, T_tr) (closure, Boltzmann tail)
    double *QDH = Qv + NL;           // [NL] ... at the HPID backward T (molecules)
    double *QDE = QDH + NL;          // [NL] ... at the EID backward T (molecules)
    double *sE = QDE + NL;           // [NL] state energies: level energies or electronic terms
    double *xs = sE + NL;            // [L] solution

    const double Ttr = cells.T_tr[c], Tv = cells.T_v[c], ne = cells.n_e[c];
    const double *Nc = cells.N + (int64_t)c * S;
    const double Ns = Nc[R.species];
    const CellSpecies q = cs[(int64_t)c * S + R.species];
    const int64_t orow = ((int64_t)c * cr.n + r) * cr.LS;
    if (!(Ns > 0.0) || !(q.lnNQ > -INFINITY)) {
        // no atoms in the cell: no level populations (the lines are skipped)
        for (int j = lane; j < NL; j += 64) {
            cr.pop[orow + j] = 0.0;
            cr.lnd[orow + j] = 0.0;
        }
        return;
    }
    double NM = 0.0;   // heavy colliders
    for (int s = 0; s < S; ++s) NM += cr.collider_w[s] * Nc[s];
    const double Nion = R.ion >= 0 ? Nc[R.ion] : 0.0;
    double Tm[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) Tm[k] = rate_temperature(R.texp[k], Ttr, Tv);
    const double *lE = sp.lev_E + R.lev0, *lg = sp.lev_g + R.lev0;

    if (!mol) {
        for (int j = lane; j < NL; j += 64) {
            QH[j] = lg[j] * exp(-kC2 * lE[j] / Tm[1]);
            QE[j] = lg[j] * exp(-kC2 * lE[j] / Tm[3]);
            Qv[j] = lg[j] * exp(-kC2 * lE[j] / Tv);
            sE[j] = lE[j];
        }
    } else {
        for (int j = 0; j < NL; ++j) {   // wave-uniform: the (v, J) sums use every lane
            const int64_t e = R.e0 + j;
            double o[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            if (R.diss_x >= 0) {
                const double T4[4] = {Tm[1], Tm[3], Tm[9], Tm[11]};
                mol_state_q<4>(sp, e, Tv, Ttr, T4, lane, o);
            } else {
                const double T2[2] = {Tm[1], Tm[3]};
                mol_state_q<2>(sp, e, Tv, Ttr, T2, lane, o);
            }
            const double qv = o[0], qh = o[1], qe = o[2], qdh = o[3], qde = o[4];
            if (lane == 0) {
                QH[j] = qh;
                QE[j] = qe;
                Qv[j] = qv;
                QDH[j] = qdh;
                QDE[j] = qde;
                sE[j] = sp.el_T[e];
            }
        }
    }
    __syncthreads();

    // Collisional rate K(i -> m) in s^-1, stored transposed at M[m][i]: row i
    // of R then holds the gains of level i (R[i][j] = K(j -> i)) and column i
    // the losses of level i.  Row 0 is overwritten by the closure below, after
    // the losses have been summed.
    for (int e = lane; e < L * L; e += 64) {
        const int i = e / L, m = e - i * L;
        double v = 0.0;
        if (i != m)
            v = k_exc(R.hpie, L, i, m, Tm[0], Tm[1], QH) / kAvogadro * NM +
                k_exc(R.eie, L, i, m, Tm[2], Tm[3], QE) / kAvogadro * ne;
        M[m * ld + i] = v;
    }
    __syncthreads();

    double loss = 0.0;
    const int i = lane;
    if (i >= 1 && i < L) {
        for (int m = 0; m < L; ++m)
            if (m != i) loss += M[m * ld + i];
        // spontaneous emission to lower states, escape factor 0 above nu_cut
        for (int m = 0; m < i; ++m) loss += (sE[i] - sE[m] > R.nu_cut ? 0.0 : 1.0) * R.A[i * L + m];
        if (!mol) {
            loss += arrhenius(R.eii + 3 * i, Tm[4]) / kAvogadro * ne;
            if (R.partner >= 0) loss += arrhenius(R.ce + 3 * i, Tm[6]) / kAvogadro * Nc[R.partner_ion];
        } else if (R.diss_x >= 0) {
            loss += arrhenius(R.hpid + 3 * i, Tm[8]) / kAvogadro * NM + arrhenius(R.eid + 3 * i, Tm[10]) / kAvogadro * ne;
        }
    }
    __syncthreads();
    if (i == 0) {
        // closure: sum of all levels = N, the levels above L-1 in Boltzmann
        // ratio with level L-1
        double *row = M;
        for (int j = 0; j < L; ++j) row[j] = 1.0;
        double t = 0.0;
        for (int p = L; p < NL; ++p) t += Qv[p] / Qv[L - 1];
        row[L - 1] = 1.0 + t;
        row[L] = Ns;
    } else if (i < L) {
        double *row = M + i * ld;
        row[i] = -loss;
        for (int j = i + 1; j < L; ++j) row[j] += (sE[j] - sE[i] > R.nu_cut ? 0.0 : 1.0) * R.A[j * L + i];
        if (mol) {
            // three-body recombination of the dissociation products into the
            // state, k_b = [k_D Q_i / (Q_X Q_Y)]_{T_b} (h^2/(2 pi mu k T_b))^{3/2}
            // e^{c2 E_diss / T_b}, by heavy particles and by electrons
            double src = 0.0;
            if (R.diss_x >= 0) {
                const double NXY[2] = {NM, ne};
                for (int d = 0; d < 2; ++d) {
                    const double Tb = Tm[9 + 2 * d];
                    const double *tab = d == 0 ? R.hpid : R.eid;
                    const double Qi = d == 0 ? QDH[i] : QDE[i];
                    const double Vmu = pow(kPlanck * kPlanck / (2.0 * kPi * R.mu * kBoltz * Tb), 1.5);
                    const double kb = arrhenius(tab + 3 * i, Tb) * Qi /
                                      (product_q(sp, R.x_lev0, R.nx_lev, R.Q_x, Tb) *
                                       product_q(sp, R.y_lev0, R.ny_lev, R.Q_y, Tb)) *
                                      Vmu * exp(kC2 * R.E_diss / Tb);
                    src += kb / kAvogadro * Nc[R.diss_x] * Nc[R.diss_y] * NXY[d];
                }
            }
            row[L] = -src;
        } else {
        // sources from outside the atom: three-body recombination of the ion,
        // k_rec = [k_EII Q_i / (Q_ion e^{-c2 E_ion/T} Q_e)]_{T_b}, Q_e the free
        // electron's 2 (2 pi m_e k T / h^2)^{3/2}; charge exchange of the ion with
        // the partner atom, k_b = [k_CE Q_i Q_B+ / (Q_A+ Q_B)]_{T_b}
        const double Tb = Tm[5];
        const double V = pow(kPlanck * kPlanck / (2.0 * kPi * kMe * kBoltz * Tb), 1.5);
        const double krec = arrhenius(R.eii + 3 * i, Tb) * (lg[i] * exp(-kC2 * lE[i] / Tb)) /
                            (R.Q_ion * exp(-kC2 * R.E_ion / Tb) * (2.0 / V));
        double src = krec / kAvogadro * Nion * ne * ne;
        if (R.partner >= 0) {
            const double Tc = Tm[7];
            double QB = 0.0;
            for (int k = 0; k < R.pn_lev; ++k)
                QB += sp.lev_g[R.plev0 + k] * exp(-kC2 * sp.lev_E[R.plev0 + k] / Tc);
            const double QBp = R.pQ_ion * exp(-kC2 * R.pE_ion / Tc);
            const double QAp = R.Q_ion * exp(-kC2 * R.E_ion / Tc);
            const double kb = arrhenius(R.ce + 3 * i, Tc) * (lg[i] * exp(-kC2 * lE[i] / Tc)) * QBp / (QAp * QB);
            src += kb / kAvogadro * Nion * Nc[R.partner];
        }
        row[L] = -src;
        }
    }
    __syncthreads();

    // LU with partial pivoting (largest magnitude, first on ties), the right
    // hand side carried along as column L.  A NaN entry ranks below every
    // number, so the wave always agrees on one pivot row in [k, L).
    for (int k = 0; k < L; ++k) {
        double v = -1.0;
        if (lane >= k && lane < L) {
            const double a = fabs(M[lane * ld + k]);
            v = a == a ? a : -0.5;
        }
        int p = lane;
        for (int o = 32; o > 0; o >>= 1) {
            const double v2 = __shfl_xor(v, o);
            const int p2 = __shfl_xor(p, o);
            if (v2 > v || (v2 == v && p2 < p)) {
                v = v2;
                p = p2;
            }
        }
        if (p != k)
            for (int j = lane; j <= L; j += 64) {
                const double a = M[k * ld + j];
                M[k * ld + j] = M[p * ld + j];
                M[p * ld + j] = a;
            }
        __syncthreads();
        if (lane > k && lane < L) {
            double *row = M + lane * ld;
            const double f = row[k] / M[k * ld + k];
            for (int j = k + 1; j <= L; ++j) row[j] -= f * M[k * ld + j];
        }
        __syncthreads();
    }
    for (int k = L - 1; k >= 0; --k) {
        const double xk = M[k * ld + L] / M[k * ld + k];
        if (lane < k) M[lane * ld + L] -= M[lane * ld + k] * xk;
        if (lane == k) xs[k] = xk;
        __syncthreads();
    }

    // populations and their ln departures from the Boltzmann populations the
    // line setup uses: ln(N/Q) + ln g - c2 E / T_v for an atomic level,
    // ln(N/Q) + ln Q_e(T_v, T_tr) for a molecular state (-inf for a
    // population <= 0)
    const double bv = kC2 / Tv;
    for (int j = lane; j < NL; j += 64) {
        const double pj = j < L ? xs[j] : xs[L - 1] * Qv[j] / Qv[L - 1];
        const double lnB = mol ? q.lnNQ + log(Qv[j]) : (q.lnNQ + log(lg[j])) - bv * lE[j];
        cr.pop[orow + j] = pj;
        cr.lnd[orow + j] = pj > 0.0 ? log(pj) - lnB : (pj <= 0.0 ? -INFINITY : pj);
    }
}

}  // namespace

hipError_t launch_cr(const DevSpecies &sp, const DevCells &cells, const DevCR &cr, int32_t max_l,
                     int32_t max_lev, const CellSpecies *cs, hipStream_t st)
{
    if (cr.n < 1 || cells.n_cells < 1) return hipSuccess;
    const size_t lds = ((size_t)max_l * row_stride(max_l) + 6 * (size_t)max_lev + max_l) * sizeof(double);
    hipLaunchKernelGGL(cr_kernel, dim3((unsigned)cells.n_cells * (unsigned)cr.n), dim3(64), lds, st, sp,
                       cells, cr, cs);
    return hipGetLastError();
}

}  // namespace lrt

"""Scaling-exponent validation in the form of the paper's Table I
(arXiv:1710.10420, Sec. III): sets of five runs with five fixed seeds, in
single and in double precision, of a 2048^2 and a 128^3 lattice; the
exponents mu (rho ~ eta^mu) and nu (gamma v ~ eta^nu) of Eq. (9) are fitted
over the records with ln(eta) > 2.58 and reported as the mean over the five
runs with its one-sigma statistical error (standard error of the mean).

The paper does not give the era, the wall width, the time step or the final
time of these runs; the defaults below are this library's workload
conventions (radiation era m = 1, W0 = 10, deta = 0.25 in 2D and 0.2 in 3D,
runs to eta = N/2), so the numbers are comparable with the paper's in kind,
not digit for digit.

    python -m paper_1710_10420_amd.validation
"""
import json
import math
import sys

LN_ETA_MIN = 2.58          # Table I: points beyond log(eta) = 2.58 (natural log)
SEEDS = (1, 2, 3, 4, 5)

CASES = (
    dict(name="2048^2", shape=(2048, 2048), deta=0.25, diag_every=16),
    dict(name="128^3", shape=(128, 128, 128), deta=0.2, diag_every=5),
)


def run_exponents(prs, case, seed, precision, tuned, m=1.0, W0=10.0):
    """One run from the seeded field to eta = N/2; returns (mu, nu).  The
    first run of a (lattice, precision) pair is autotuned and its tiling and
    steps per pass are reused through `tuned`."""
    shape = case["shape"]
    eta_end = shape[0] / 2.0
    steps = int(round((eta_end - 1.0) / case["deta"]))
    p = prs.make_params(shape, deta=case["deta"], m=m, W0=W0, diag_every=case["diag_every"],
                        precision=precision)
    sim = prs.Sim(p, seed=seed)
    key = (case["name"], precision)
    if key not in tuned:
        prs.prs_autotune(sim.ctx, None, 0)
        tuned[key] = (sim.tiling(), sim.time_blocking())
    sim.set_tiling(*tuned[key][0])
    sim.set_time_blocking(tuned[key][1])
    recs = sim.step_n(steps)
    recs.append(sim.wall_stats())
    sim.close()
    return prs.prs_fit_scaling(recs, math.exp(LN_ETA_MIN), math.inf)


def mean_err(values):
    n = len(values)
    mean = sum(values) / n
    var = sum((v - mean) ** 2 for v in values) / (n - 1) if n > 1 else 0.0
    return mean, math.sqrt(var / n)


def scaling_table(prs, cases=CASES, seeds=SEEDS):
    """{case: {precision: {"mu": (mean, err), "nu": (mean, err), "runs": [(mu, nu), ...]}}}"""
    out = {}
    tuned = {}
    for case in cases:
        row = {}
        for label, precision in (("single", prs.PRS_F32), ("double", prs.PRS_F64)):
            runs = [run_exponents(prs, case, s, precision, tuned) for s in seeds]
            row[label] = {"mu": mean_err([r[0] for r in runs]), "nu": mean_err([r[1] for r in runs]),
                          "runs": runs}
        out[case["name"]] = row
    return out


def main():
    from paper_1710_10420_amd import prs
    table = scaling_table(prs)
    for name, row in table.items():
        for label, r in row.items():
            print("%-7s %-6s mu = %.4f +- %.4f   nu = %.4f +- %.4f" % (
                name, label, r["mu"][0], r["mu"][1], r["nu"][0], r["nu"][1]))
    print(json.dumps(table))
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Fixed short workloads for kernel profiling (rocprofv3 kernel traces and
hardware-counter passes).

    python -m paper_1710_10420_amd.profile_step --workload 2d8192 --steps 40

Runs `steps` plain leapfrog steps (no diagnostics) of the chosen lattice in
its default tiling, then `copies` copies of a 256 MiB float32 buffer with
torch (a plain copy kernel of known size: 256 MiB read + 256 MiB written per
dispatch), which calibrates the byte counters against a kernel whose traffic
is known exactly.

    python -m paper_1710_10420_amd.profile_step --ensemble 0 --ensemble-settings \
        "1024x1024=1,16,1,8;2048x2048=2,64,1,8;..."

runs the seeded 64-realisation ensemble (master seed 2017) instead, in the
given batch mode with the given tiling and steps per pass per lattice, once
untimed and then `ensemble-runs` times, before the copies.
"""
import argparse
import sys

import torch

from paper_1710_10420_amd import prs

WORKLOADS = {
    "2d8192": dict(shape=(8192, 8192), deta=0.25, m=2.0, W0=10.0),
    "3d1024": dict(shape=(1024, 1024, 1024), deta=0.2, m=1.0, W0=10.0),
    "2d2048": dict(shape=(2048, 2048), deta=0.25, m=1.0, W0=10.0),
    "3d256": dict(shape=(256, 256, 256), deta=0.2, m=1.0, W0=10.0),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="2d8192", choices=sorted(WORKLOADS))
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--copies", type=int, default=10)
    ap.add_argument("--adjoint", action="store_true", help="also run an adjoint")
    ap.add_argument("--adjoint-steps", type=int, default=64, help="steps of the adjoint run")
    ap.add_argument("--ckpt", type=int, default=64, help="checkpoint interval of the adjoint run")
    ap.add_argument("--tiling", default=None, help="vec,rows,ty (default: the library default)")
    ap.add_argument("--steps-per-pass", type=int, default=None, help="steps per forward pass")
    ap.add_argument("--adjoint-tiling", default=None, help="vec,rows,ty of the reverse sweep")
    ap.add_argument("--adjoint-steps-per-pass", type=int, default=None, help="steps per reverse pass")
    ap.add_argument("--ensemble", type=int, default=None, help="batch mode of an ensemble run instead")
    ap.add_argument("--ensemble-settings", default="",
                    help="lattice=vec,rows,ty,steps_per_pass entries separated by ';' (lattice as NxN or NxNxN)")
    ap.add_argument("--ensemble-runs", type=int, default=2)
    args = ap.parse_args()
    if args.ensemble is not None:
        ensemble(args.ensemble, args.ensemble_settings, args.ensemble_runs)
        copies(args.copies)
        print("done", flush=True)
        return 0
    w = WORKLOADS[args.workload]
    p = prs.make_params(w["shape"], deta=w["deta"], m=w["m"], W0=w["W0"])
    sim = prs.Sim(p, seed=1)
    if args.tiling:
        sim.set_tiling(*[int(v) for v in args.tiling.split(",")])
    if args.steps_per_pass:
        sim.set_time_blocking(args.steps_per_pass)
    if args.adjoint_tiling:
        prs.prs_set_adjoint_tiling(sim.ctx, *[int(v) for v in args.adjoint_tiling.split(",")])
    if args.adjoint_steps_per_pass:
        prs.prs_set_adjoint_time_blocking(sim.ctx, args.adjoint_steps_per_pass)
    print("workload", args.workload, "tiling", sim.tiling(), "steps/pass", sim.time_blocking(), flush=True)
    sim.step_n(args.steps, diag=False)
    torch.cuda.synchronize()
    if args.adjoint:
        nb = prs.prs_adjoint_workspace_bytes(p, args.adjoint_steps, args.ckpt)
        work = torch.empty(nb, dtype=torch.uint8, device="cuda")
        g = torch.empty_like(sim.phi_a)
        prs.prs_adjoint(sim.ctx, args.adjoint_steps, args.ckpt, work.data_ptr(), nb, g.data_ptr(), None)
        torch.cuda.synchronize()
    copies(args.copies)
    print("done", flush=True)
    return 0


def copies(n):
    src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(n):
        dst.copy_(src)
    torch.cuda.synchronize()


def ensemble(mode, settings, runs):
    from paper_1710_10420_amd.inputs import ensemble_draw
    table = {}
    for entry in filter(None, settings.split(";")):
        key, val = entry.split("=")
        v = [int(x) for x in val.split(",")]
        table[tuple(int(n) for n in key.split("x"))] = ((v[0], v[1], v[2]), v[3])
    items = ensemble_draw(2017)
    specs = [dict(shape=(it["N"],) * it["ndim"], deta=it["deta"], m=it["m"], W0=it["W0"], nsteps=it["steps"],
                  diag_every=64 if it["ndim"] == 2 else 50, seed=it["seed"]) for it in items]
    b = prs.Batch(specs)
    for r, sp in enumerate(specs):
        if sp["shape"] in table:
            til, T = table[sp["shape"]]
            b.set_time_blocking(r, 1)
            b.set_tiling(r, *til)
            b.set_time_blocking(r, T)
    b.set_mode(mode)
    print("ensemble mode", mode, {"x".join(map(str, k)): v for k, v in table.items()}, flush=True)
    for _ in range(1 + runs):
        b.run()
    torch.cuda.synchronize()
    b.close()


if __name__ == "__main__":
    sys.exit(main())

"""Time one hot kernel of the library in isolation, for profiling and tuning.

    python -m paper_1205_2933_amd.kernel_bench --kernel dslash --prec f32 --nrhs 12

Sets up a handle on the given lattice with seeded random data (links and
basis vectors drawn with torch; their values do not change the memory traffic),
launches the kernel through mgdwf_time_kernel on the library stream and prints
one JSON line with the mean launch time and the algorithmic bandwidth.
``--kernel copy`` times a plain device-to-device copy of one fine field of the
given precision; it is the reference for hardware traffic counters.

Algorithmic bytes per launch (complex numbers of b bytes, V5 = V4 Ls):
  dslash    nrhs (2 x 12 V5) b + 36 V4 b           (read in, write out, links)
  restrict  nrhs 12 V5 b + Nv 12 V5 b              (read x, read the basis)
  prolong   nrhs 12 V5 b + Nv 12 V5 b
  coarse    9 (2Nv)^2 Vc s + nrhs 2 (2 Nv Vc) b    (s = bytes per stored entry)
            33 offsets instead of 9 with --squared (A_c = P^+ D^+D P; in 2D
            the 9 nonzero ones of its 33-offset store)
With --model 2d the lattice is the 2D U(1) one (--L2 Lx Ly, 2 spins, U(1)
links: 12 becomes 2 and 36 V4 becomes 2 V2; blocks --block2 bx by; the
coarse operator is the squared one).
"""

from __future__ import annotations

import argparse
import json

import torch

from . import _lib as mg

HBM_PEAK_GBS = 8000.0
KERNELS = {"dslash": mg.MGDWF_K_DSLASH, "restrict": mg.MGDWF_K_RESTRICT, "prolong": mg.MGDWF_K_PROLONG,
           "coarse": mg.MGDWF_K_COARSE}
BYTES = {"f64": 16, "f32": 8, "f16": 4, "bf16": 4}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernel", choices=sorted(KERNELS) + ["copy"], default="dslash")
    ap.add_argument("--prec", choices=sorted(BYTES), default="f32")
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--L", type=int, nargs=4, default=(16, 16, 16, 32))
    ap.add_argument("--Ls", type=int, default=16)
    ap.add_argument("--block", type=int, nargs=4, default=(4, 4, 4, 4))
    ap.add_argument("--nvec", type=int, default=24)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--tiling", type=int, default=-1, help="FP32 Dslash tiling id (mgdwf_set_tiling), -1 = default")
    ap.add_argument("--model", choices=("4d", "2d"), default="4d")
    ap.add_argument("--L2", type=int, nargs=2, default=(20, 20))
    ap.add_argument("--block2", type=int, nargs=2, default=(4, 4))
    ap.add_argument("--squared", action="store_true", help="time A_c = P^+ D^+D P (33 offsets) for --kernel coarse")
    ap.add_argument("--coarse-tile", type=int, default=-1,
                    help="MFMA shape of the 16-bit D_c apply: 0 = 16x16x16, 1 = 16x16x32, -1 = default")
    args = ap.parse_args(argv)

    dev = torch.device("cuda:0")
    two_d = args.model == "2d"
    L = (args.L2[0], args.L2[1], 1, 1) if two_d else tuple(args.L)
    Ls = args.Ls
    block = (args.block2[0], args.block2[1], 1, 1) if two_d else tuple(args.block)
    V4 = L[0] * L[1] * L[2] * L[3]
    V5 = V4 * Ls
    nsc = 2 if two_d else 12          # complex numbers per 5D site
    nlink = 2 if two_d else 36        # complex numbers of links per 4D (2D) site
    b = BYTES[args.prec]
    g = torch.Generator(device=dev)
    g.manual_seed(args.seed)

    if args.kernel == "copy":
        dt = torch.complex128 if args.prec == "f64" else torch.complex64
        x = torch.randn(12 * V5 * args.nrhs, dtype=dt, device=dev, generator=g)
        y = torch.empty_like(x)
        for _ in range(2):
            y.copy_(x)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.iters):
            y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.iters
        nbytes = 2 * x.numel() * x.element_size()
        print(json.dumps({"kernel": "copy", "prec": args.prec, "bytes": nbytes, "us": ms * 1e3,
                          "GBs": nbytes / (ms * 1e-3) / 1e9}), flush=True)
        return

    if two_d:
        h = mg.Handle2D(args.L2, Ls, 1.0, 0.01)
        U = torch.exp(1j * 2 * torch.pi * torch.rand(2 * V4, dtype=torch.float64, device=dev, generator=g))
    else:
        h = mg.Handle(L, Ls, 1.8, 0.001)
        U = torch.randn(36 * V4, dtype=torch.complex128, device=dev, generator=g)
    mg.mgdwf_set_gauge(h, U.contiguous())
    del U
    if not two_d:
        mg.mgdwf_set_tiling(h, args.tiling)
    squared = args.squared or two_d
    if args.kernel != "dslash":
        V = torch.randn(nsc * V5 * args.nvec, dtype=torch.complex128, device=dev, generator=g)
        mg.mgdwf_set_nullvecs(h, block, V, args.nvec)
        del V
        if squared:
            mg.mgdwf_build_coarse_squared(h)
        else:
            mg.mgdwf_build_coarse(h)
            mg.mgdwf_set_coarse_tiling(h, args.coarse_tile)
    torch.cuda.synchronize()
    ms = mg.mgdwf_time_kernel(h, KERNELS[args.kernel], args.prec, args.nrhs, args.iters)
    if args.kernel == "dslash":
        nbytes = args.nrhs * 2 * nsc * V5 * b + nlink * V4 * b
    elif args.kernel in ("restrict", "prolong"):
        nbytes = (args.nrhs + args.nvec) * nsc * V5 * b
    else:
        Vc = V4 // (block[0] * block[1] * block[2] * block[3])
        n2 = 2 * args.nvec
        store = 16 if args.prec == "f64" else (8 if args.prec == "f32" else 4)
        vec = 16 if args.prec == "f64" else 8
        noff = 9 if (two_d or not squared) else 33  # the 2D store's z and t offsets are zero: not algorithmic
        nbytes = noff * n2 * n2 * Vc * store + args.nrhs * 2 * n2 * Vc * vec
    gbs = nbytes / (ms * 1e-3) / 1e9
    print(json.dumps({"kernel": args.kernel, "model": args.model, "squared": squared, "prec": args.prec,
                      "nrhs": args.nrhs, "L": L, "Ls": Ls,
                      "tiling": args.tiling, "coarse_tile": args.coarse_tile, "bytes": nbytes,
                      "us": ms * 1e3, "GBs": gbs, "frac_hbm_peak": gbs / HBM_PEAK_GBS}), flush=True)
    h.close()


if __name__ == "__main__":
    main()

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
    ap.add_argument("--coarse-tile", type=int, default=-1,
                    help="MFMA shape of the 16-bit D_c apply: 0 = 16x16x16, 1 = 16x16x32, -1 = default")
    args = ap.parse_args(argv)

    dev = torch.device("cuda:0")
    L, Ls = tuple(args.L), args.Ls
    V4 = L[0] * L[1] * L[2] * L[3]
    V5 = V4 * Ls
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

    h = mg.Handle(L, Ls, 1.8, 0.001)
    U = torch.randn(36 * V4, dtype=torch.complex128, device=dev, generator=g)
    mg.mgdwf_set_gauge(h, U)
    del U
    mg.mgdwf_set_tiling(h, args.tiling)
    if args.kernel != "dslash":
        V = torch.randn(12 * V5 * args.nvec, dtype=torch.complex128, device=dev, generator=g)
        mg.mgdwf_set_nullvecs(h, args.block, V, args.nvec)
        del V
        mg.mgdwf_build_coarse(h)
        mg.mgdwf_set_coarse_tiling(h, args.coarse_tile)
    torch.cuda.synchronize()
    ms = mg.mgdwf_time_kernel(h, KERNELS[args.kernel], args.prec, args.nrhs, args.iters)
    if args.kernel == "dslash":
        nbytes = args.nrhs * 24 * V5 * b + 36 * V4 * b
    elif args.kernel in ("restrict", "prolong"):
        nbytes = (args.nrhs + args.nvec) * 12 * V5 * b
    else:
        Vc = V4 // (args.block[0] * args.block[1] * args.block[2] * args.block[3])
        n2 = 2 * args.nvec
        store = 16 if args.prec == "f64" else (8 if args.prec == "f32" else 4)
        vec = 16 if args.prec == "f64" else 8
        nbytes = 9 * n2 * n2 * Vc * store + args.nrhs * 2 * n2 * Vc * vec
    gbs = nbytes / (ms * 1e-3) / 1e9
    print(json.dumps({"kernel": args.kernel, "prec": args.prec, "nrhs": args.nrhs, "L": L, "Ls": Ls,
                      "tiling": args.tiling, "coarse_tile": args.coarse_tile, "bytes": nbytes,
                      "us": ms * 1e3, "GBs": gbs, "frac_hbm_peak": gbs / HBM_PEAK_GBS}), flush=True)
    h.close()


if __name__ == "__main__":
    main()

"""Small program for hardware-counter runs: one end-to-end step (set-up,
factorisation, GMRES solve) of a workload on one precision path, followed by
a plain device-to-device copy of a known size that calibrates the FETCH_SIZE
/ WRITE_SIZE counters (bytes the copy must read and write).

    rocprofv3 --pmc FETCH_SIZE --kernel-trace -d <dir> -- \
        python -m paper_1408_4495_amd.profile_probe --workload c2 --precision mixed
"""
import argparse
import os
import sys


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--copy-mib", type=int, default=256)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch
    import synth
    from paper_1408_4495_amd import lsp

    w = synth.workload(args.workload)
    dev = torch.device("cuda:0")
    m = torch.tensor(w["m"], dtype=torch.float64, device=dev)
    u = torch.tensor(w["uI"], dtype=torch.complex128, device=dev)
    plan = lsp.Plan(w["n"], w["d"], max_nrhs=u.shape[0], precision=args.precision)
    pb = lsp.Problem(plan, w["omega"], m)
    pb.factor()
    _, info, st = pb.solve(u)
    torch.cuda.synchronize()
    nbytes = args.copy_mib << 20
    a = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"probe done: status {st}, iters {[i['iters'] for i in info]}, copy {nbytes} bytes", flush=True)


if __name__ == "__main__":
    main()

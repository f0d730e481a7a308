"""Workload for HBM-traffic counters of the root-level MTTKRP.

Runs, on the current HIP stream: three plain device copies of 256 MiB (the
calibration: each moves exactly 256 MiB in and 256 MiB out), then one
root-level MTTKRP per mode of the NELL-2-shaped tensor (rank 35, FP32, one
tree rooted at each mode, the others by descending length: the launch
configuration of cpd_als).  Meant to be
run under `rocprofv3 --pmc FETCH_SIZE` and `--pmc WRITE_SIZE`; the counter
values of the copy kernels give the scale factor applied to the MTTKRP's.

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT -o run -- \
        python -m paper_1812_05961_amd.traffic_probe
"""
import torch

from . import cpd, synth


def main():
    cpd.lib()
    dev = torch.device("cuda:0")
    n = 64 << 20  # floats: 256 MiB
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    x = synth.make_config("nell2", device=dev)
    inds = x.inds.to(torch.int32)
    R, ld = 35, 36
    g = torch.Generator(device="cuda").manual_seed(1)
    facs = []
    for d in x.dims:
        f = torch.zeros((d, ld), dtype=torch.float32, device=dev)
        f[:, :R] = torch.rand((d, R), device=dev, generator=g)
        facs.append(f)
    for mode in range(3):
        rest = sorted([q for q in range(3) if q != mode], key=lambda q: (-x.dims[q], q))
        c = cpd.csf_build(inds, x.vals, x.dims, [mode] + rest)
        out = torch.empty((x.dims[mode], ld), device=dev)
        cpd.mttkrp(c, facs, mode, out=out, rank=R)
        torch.cuda.synchronize()
        c.free()
    print("traffic probe done", flush=True)


if __name__ == "__main__":
    main()

"""Plain device copy of a known size, for scaling HBM traffic counters.

Run under `rocprofv3 --pmc FETCH_SIZE` (then `WRITE_SIZE`): each of the
`--reps` dispatches of torch's copy kernel moves exactly `--mib` MiB in and
`--mib` MiB out, so counter / expected gives the factor by which a counter
over- or under-reports bytes on this device.
"""
import argparse


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    import torch

    n = args.mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(args.reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {args.reps} x {args.mib} MiB", flush=True)


if __name__ == "__main__":
    main()

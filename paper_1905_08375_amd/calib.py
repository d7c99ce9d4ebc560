"""Reference copy of a known size, used to calibrate the rocprofv3 memory
counters (FETCH_SIZE / WRITE_SIZE) against exactly known traffic:
`python -m paper_1905_08375_amd.calib` copies a 256 MiB FP32 buffer 20 times."""
import torch


def main(mib: int = 256, reps: int = 20):
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB x {reps}", flush=True)


if __name__ == "__main__":
    main()

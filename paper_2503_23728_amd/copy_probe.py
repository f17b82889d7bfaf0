"""A plain device-to-device copy of known size (64 MiB, three times).

Used to calibrate the FETCH_SIZE / WRITE_SIZE hardware counters: the ratio
of the bytes a copy moves to what the counters report scales the counters of
the path's kernels to HBM bytes."""
import torch

N_BYTES = 64 * 1024 * 1024

if __name__ == "__main__":
    a = torch.ones(N_BYTES // 4, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {N_BYTES} bytes x3")

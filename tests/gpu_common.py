"""Helpers shared by the GPU parity tests (HIP path vs the CPU oracle)."""
import math

import numpy as np

# Results the two sides must reproduce bit for bit: integers, flags, the
# selection, and every value computed by exact operations in a fixed order
# (min/max, the value range, the tree sums of squared errors, delta = sqrt(12
# MSE) and 1/delta, bit-rates that are integer ratios).
EXACT_KEYS = [
    "flags", "choice", "minexp", "vmin", "vmax", "vr", "eb_abs",
    "zfp_bits", "zfp_values", "zfp_blocks", "zfp_nsb_total", "zfp_sse", "zfp_mse",
    "zfp_bitrate", "zfp_nsb_mean", "zfp_maxerr",
    "sz_delta", "sz_inv_delta", "sz_eb", "sz_sse", "sz_mse", "sz_maxerr",
    "sz_values", "sz_unpredictable", "chosen_eb",
    "sz_huffman_bits", "sz_huffman_bitrate", "zfp_ec_points", "zfp_ec_nsb2",
]
# Results that go through log2 / log10 (device and host math libraries may
# differ in the last bits): 1e-9 relative.
REL_KEYS = ["zfp_psnr", "sz_entropy", "sz_bitrate", "sz_psnr_model", "sz_psnr_measured"]
REL_TOL = 1e-9


def same_float(a, b):
    if isinstance(a, float) and math.isnan(a):
        return isinstance(b, float) and math.isnan(b)
    return a == b


def assert_matches_oracle(gpu: dict, orc: dict, label=""):
    bad = []
    for k in EXACT_KEYS:
        if not same_float(gpu[k], orc[k]):
            bad.append("%s: gpu %r oracle %r" % (k, gpu[k], orc[k]))
    for k in REL_KEYS:
        a, b = gpu[k], orc[k]
        if math.isinf(a) or math.isinf(b) or a == b:
            if a != b:
                bad.append("%s: gpu %r oracle %r" % (k, a, b))
            continue
        if abs(a - b) > REL_TOL * max(abs(a), abs(b)):
            bad.append("%s: gpu %r oracle %r" % (k, a, b))
    assert not bad, "%s\n  " % label + "\n  ".join(bad)


def is_tie(orc: dict) -> bool:
    """Selections whose bit-rates agree to 1e-9 relative are ties."""
    a, b = orc["sz_bitrate"], orc["zfp_bitrate"]
    return abs(a - b) <= 1e-9 * max(abs(a), abs(b), 1e-300)


def debug_buffers(torch, nblk, nd, device="cuda"):
    size = 4 ** nd
    return {
        "codes": torch.zeros(max(1, nblk * size), dtype=torch.int16, device=device),
        "zfp_bits": torch.zeros(max(1, nblk), dtype=torch.int32, device=device),
        "zfp_sse": torch.zeros(max(1, nblk), dtype=torch.float64, device=device),
        "zfp_emax": torch.zeros(max(1, nblk), dtype=torch.int32, device=device),
        "sz_sse": torch.zeros(max(1, nblk), dtype=torch.float64, device=device),
        "hist": torch.zeros(65536, dtype=torch.int32, device=device),
    }


def debug_to_numpy(d, nblk, nd):
    size = 4 ** nd
    return {
        "codes": d["codes"].cpu().numpy().view(np.uint16)[: nblk * size],
        "zfp_bits": d["zfp_bits"].cpu().numpy().view(np.uint32)[:nblk],
        "zfp_sse": d["zfp_sse"].cpu().numpy()[:nblk],
        "zfp_emax": d["zfp_emax"].cpu().numpy()[:nblk],
        "sz_sse": d["sz_sse"].cpu().numpy()[:nblk],
        "hist": d["hist"].cpu().numpy().view(np.uint32),
    }

"""The surrogate peel-off recipe for the flared-disk scene (disk128): the
cylindrical domain, the pilot and validation sample sizes, the Adam schedule and
the validity thresholds.  One place for the numbers that the benchmark reports
and the full-size parity test checks.  `train_disk_surrogate` only calls the
library's entry points (sampling, training and validation run on the GPU)."""
from __future__ import annotations

DISK_DOMAIN = dict(center=(0.0, 0.0, 0.0), r_in=0.05, r_out=1.0, h0=0.1, beta=1.125, zmax_over_h=3.0)
DOMAIN_CELLS = dict(n_r=16, n_z=12)
N_TRAIN, N_VAL = 1 << 20, 1 << 17
PILOT_SEED, VAL_SEED = 101, 202
TRAIN = dict(steps=20000, batch=8192, lr=2e-3, lr_final=5e-5, seed=7, tau_cap=12.0, weight_floor=0.02)
VALIDATE = dict(max_err=0.02, floor_frac=0.3, min_count=16)


def train_disk_surrogate(ctx, timer=None, h0: float = DISK_DOMAIN["h0"]):
    """Domain, pilot samples (exact labels), training and validity mask on a
    context set up with a disk scene of scale height h0 R^1.125.  timer(fn) ->
    (result, seconds) times a step (default: untimed).  Returns (pilot_packets,
    train_report, mask_report, {step: seconds})."""
    import torch
    if timer is None:
        timer = lambda fn: (fn(), 0.0)   # noqa: E731
    ctx.surrogate_set_domain(**DOMAIN_CELLS, **dict(DISK_DOMAIN, h0=h0))
    pos = torch.zeros((N_TRAIN, 4), dtype=torch.float32, device="cuda")
    tau = torch.zeros(N_TRAIN, dtype=torch.float32, device="cuda")
    pilot, t_sample = timer(lambda: ctx.surrogate_sample(pos, tau, seed=PILOT_SEED))
    vpos = torch.zeros((N_VAL, 4), dtype=torch.float32, device="cuda")
    vtau = torch.zeros(N_VAL, dtype=torch.float32, device="cuda")
    ctx.surrogate_sample(vpos, vtau, seed=VAL_SEED)
    rep, t_train = timer(lambda: ctx.surrogate_train(pos, tau, **TRAIN))
    mrep, t_val = timer(lambda: ctx.surrogate_validate(vpos, vtau, **VALIDATE))
    return pilot, rep, mrep, {"sample_s": t_sample, "train_s": t_train, "validate_s": t_val}

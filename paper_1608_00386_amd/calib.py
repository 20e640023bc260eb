"""Set-up helpers for interaction-matrix calibration and the control matrix (Sec. 2.5-2.6).

The calibration plan sees only the deformable mirrors: a flat atmosphere contributes nothing to
a push-pull difference, so turbulence layers are left out and every realisation of the batch
carries one actuator poke.  The DM grids keep their order and sizes, contiguous from offset 0,
so actuator j of the calibration buffer is actuator j of the closed-loop DM rows.
"""

import copy

import torch

from . import wfs


def dm_config(cfg, batch=128, noise=False):
    """Calibration configuration of ``cfg``: its DM grids (layers with weight < 0) only, packed
    from offset 0, ``batch`` realisations (even: batch / 2 actuators per forward call), the
    same sensors with photon and read noise switched off unless ``noise``.  Returns (config,
    number of actuators)."""
    if batch < 2 or batch % 2:
        raise ValueError(f"batch={batch} must be even and >= 2")
    dms = [copy.deepcopy(L) for L in cfg["layers"] if L["weight"] < 0]
    if not dms:
        raise ValueError("the configuration has no DM grid (layer with weight < 0)")
    o = 0
    for L in dms:
        L["offset"] = o
        o += L["nx"] * L["ny"]
    sensors = copy.deepcopy(cfg["sensors"])
    if not noise:
        for s in sensors:
            s["photons"] = 0.0
            s["read_noise_e"] = 0.0
    out = dict(name=cfg.get("name", "cfg") + "_dm_calibration", layers=dms, sensors=sensors,
               batch=int(batch), layer_stride=(o + 63) // 64 * 64,
               lambda_ref_m=cfg["lambda_ref_m"], dt_s=cfg["dt_s"])
    return out, o


def dm_weights(cfg, per_dm, device="cuda"):
    """Per-actuator regularisation weights from one weight per DM grid (in layer order)."""
    dms = [L for L in cfg["layers"] if L["weight"] < 0]
    if len(per_dm) != len(dms):
        raise ValueError(f"{len(per_dm)} weights for {len(dms)} DM grids")
    parts = [torch.full((L["nx"] * L["ny"],), float(w)) for L, w in zip(dms, per_dm)]
    return torch.cat(parts).to(device)


def calibrate_dms(cfg, amplitude=0.1, batch=128, noise=False, step=0, seed=42, flags=0):
    """Interaction matrix [n_act][n_slopes] and reference slopes of every DM actuator of
    ``cfg`` (push-pull through the batched sensor model)."""
    ccfg, n_act = dm_config(cfg, batch=batch, noise=noise)
    with wfs.Plan(ccfg, flags=flags) as plan:
        return plan.calibrate(0, n_act, amplitude=amplitude, step=step, seed=seed)

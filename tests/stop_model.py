"""Test helper: a random early-stop network whose budgets spread over the
grid, for parity tests of the fused learned stop (the weights are not
trained; the tests check that the search stops exactly where the network
says, whatever it says)."""
import torch


def random_stop_model(nsg, ix, Qd, seed, L=64, hop=16, center=5.5):
    """Random weights on features z-scored with their own statistics (taken
    from a feature capture of the plain search at pool size L after `hop`
    expansions), output scaled so the budgets spread around 2^center
    (x2^(+-1.2)) expansions; center=None puts it at log2 of the plain
    search's mean expansion count at L, so about half the searches are cut."""
    import math
    from paper_1707_00143_amd import learned_stop as ls
    dev = Qd.device
    feats = torch.empty((Qd.shape[0], nsg.STOP_FEATURES), dtype=torch.float32, device=dev)
    nsg.search_batched(ix, Qd, k_scalar=10, L_scalar=L, opts=dict(features=feats, feature_hop=hop))
    if center is None:
        hops = torch.zeros(Qd.shape[0], dtype=torch.int64, device=dev)
        nsg.search_batched(ix, Qd, k_scalar=10, L_scalar=L, opts=dict(hops=hops))
        center = math.log2(float(hops.float().mean().item()))
    keep = ~torch.isnan(feats).any(1)
    mean, istd = nsg.column_stats(feats[keep].contiguous())
    P = ls.init_params(nsg.STOP_FEATURES, ls.HIDDEN, seed)
    Pd = torch.from_numpy(P).to(dev)
    y = ls.predict(Pd, mean, istd, feats[keep].contiguous())
    sd = float(y.std().item()) or 1.0
    Pd[-(ls.HIDDEN + 1):-1] *= 1.2 / sd
    Pd[-1] = (Pd[-1] - float(y.mean().item())) * 1.2 / sd + center
    return Pd, mean, istd

"""Workload recipes (shapes, decay, scalars) for the benchmarked configurations.

Operators are dense random first block columns F_k = N(0,1) * exp(-k / tau)
(the paper's workloads are synthetic, dense, unstructured, with Nm >> Nd);
vectors are N(0,1).  The scalars of the Hessian H = noise_prec * F^T F +
prior_prec * I follow the recipes below.
"""
SEED = 13066
STREAM_BLOCKS = 0
STREAM_M = 1
STREAM_D = 2
STREAM_MTRUE = 3
STREAM_NOISE = 4
STREAM_REQUEST0 = 100

WORKLOADS = {
    # small FP64 case the oracle finishes in well under a second
    "fp64-small": dict(Nt=32, Nd=16, Nm=64, tau=8.0, storage="f64", k=1,
                       noise_prec=1.0, prior_prec=1.0),
    # one GPU's share of the plain path, FP32-complex operator (~22 GB)
    "fp32-nt420-nd100-nm65536": dict(Nt=420, Nd=100, Nm=65536, tau=60.0, storage="f32", k=1,
                                     noise_prec=1.0, prior_prec=1.0),
    # multi right-hand-side batches on the same shapes
    "multirhs-nt420-nd100-nm65536": dict(Nt=420, Nd=100, Nm=65536, tau=60.0, ks=(8, 32, 64),
                                         storages=("f32", "bf16")),
    # regularised inverse problem solved by CG
    "cg-nt256-nd64-nm16384": dict(Nt=256, Nd=64, Nm=16384, tau=256 / 7.0, sigma=1e-2, alpha=1e-3,
                                  rtol=1e-8),
    # serving: three resident operators
    "serving-3ops": dict(ops=((128, 50, 4096), (256, 100, 16384), (420, 200, 32768))),
}

// The method's scalar hyperparameters, evaluated on the host: the softplus
// shift of the low-density initialisation, the raw-density threshold of the
// coarse free-space test, and the learning-rate schedule.
#include <cmath>

#include "common.hpp"

extern "C" {

// b = log((1 - alpha_init)^(-1/s) - 1), written as log(expm1(-log1p(-alpha_init)/s))
// so that it stays accurate for small alpha_init.
int32_t dvgo_low_density_bias(double alpha_init, double voxel, double* bias) {
    if (!bias || !(alpha_init > 0.0 && alpha_init < 1.0) || !(voxel > 0.0)) return DVGO_E_ARG;
    const double sigma_s = -std::log1p(-alpha_init) / voxel;
    *bias = std::log(std::expm1(sigma_s));
    return DVGO_OK;
}

// alpha(softplus(raw + b), step) >= tau  <=>  raw >= softplus^{-1}(-log(1-tau)/step) - b;
// the float64 value is rounded down to float32, so that a float32 comparison
// keeps every point the exact test keeps.
int32_t dvgo_coarse_raw_threshold(double tau, double step, double act_shift, float* threshold) {
    if (!threshold || !(tau > 0.0 && tau < 1.0) || !(step > 0.0) || !std::isfinite(act_shift)) return DVGO_E_ARG;
    const double sigma = -std::log1p(-tau) / step;
    const double thr = std::log(std::expm1(sigma)) - act_shift;
    float t32 = static_cast<float>(thr);
    if (static_cast<double>(t32) > thr) t32 = std::nextafter(t32, -INFINITY);
    *threshold = t32;
    return DVGO_OK;
}

// lr = base_lr * decay^(it / decay_steps).
int32_t dvgo_lr_at(double base_lr, int64_t it, int64_t decay_steps, double decay, double* lr) {
    if (!lr || !(base_lr >= 0.0) || it < 0 || decay_steps <= 0 || !(decay > 0.0)) return DVGO_E_ARG;
    *lr = base_lr * std::pow(decay, static_cast<double>(it) / static_cast<double>(decay_steps));
    return DVGO_OK;
}

// Vertices per axis before checkpoint k of K: the voxel count starts at
// 1/2^K of the final one and doubles at every checkpoint, so
// floor((n_final^3 / 2^(K-k))^(1/3)) (a cube root within 1e-9 of an integer
// counts as that integer).
int32_t dvgo_pg_resolution(int32_t n_final, int32_t n_checkpoints, int32_t k, int32_t* n) {
    if (!n || n_final < 2 || n_checkpoints < 0 || k < 0 || k > n_checkpoints) return DVGO_E_ARG;
    const double x = std::cbrt(std::pow(static_cast<double>(n_final), 3.0) / std::ldexp(1.0, n_checkpoints - k));
    const int32_t v = static_cast<int32_t>(std::floor(x + 1e-9));
    *n = v < 2 ? 2 : v;
    return DVGO_OK;
}

}  // extern "C"

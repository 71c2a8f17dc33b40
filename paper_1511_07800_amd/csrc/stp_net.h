// Learned warm start for the pressure solve: a 3-level 3-D convolutional
// network (16/32/64 channels, 3x3x3 kernels) evaluated and trained with
// BF16 MFMA kernels accumulating in FP32.  Internal interface used by the
// C ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace stp {

struct NetLayer {
    int cin, cout;          // padded to multiples of 16
    int cin_logical, cout_logical;
    int level;              // 0 full grid, 1 half, 2 quarter
    long long w_off, b_off; // offsets in the FP32 parameter vector
    long long wb_off;       // offset in the BF16 weight arrays
};

class NetModel {
public:
    static constexpr int kLayers = 6;
    // bytes of device workspace for a grid (training adds the backward buffers)
    static size_t workspace_bytes(int nx, int ny, int nz, bool training);
    static bool grid_ok(int nx, int ny, int nz);

    // idx2, idy2, idz2: 1/dx^2, 1/dy^2, 1/dz^2 of the grid (for the residual input)
    NetModel(int nx, int ny, int nz, double idx2, double idy2, double idz2, bool training, void* ws,
             hipStream_t s);

    long long param_count() const { return nparam_; }
    float* params() { return P_; }
    float* grads() { return G_; }
    const NetLayer& layer(int l) const { return L_[l]; }

    hipError_t init_params(uint64_t seed);
    hipError_t sync();  // BF16 copies from the FP32 master weights; Adam state reset
    // p_guess = p_prev + s_r y(b, p_prev); all FP64 device arrays of nx*ny*nz
    hipError_t predict(const double* b, const double* p_prev, double* p_guess);
    // forward + MSE loss against (p_next - p_prev)/s_r + backward into grads();
    // Adam update with lr when lr > 0.  *loss_dev receives the loss (device).
    hipError_t train_step(const double* b, const double* p_prev, const double* p_next, float lr, double* loss_dev);

private:
    hipError_t normalise(const double* b, const double* p_prev);
    hipError_t forward();
    hipError_t backward();
    hipError_t convert_weights();

    int nx_[3], ny_[3], nz_[3];
    long long nv_[3];
    double D_, idx2_, idy2_, idz2_;
    bool training_;
    // channels per cell of the input tensor X: training's weight gradient of
    // the first layer reads 16, inference only the 8 the first layer uses
    int xstride() const { return training_ ? 16 : 8; }
    hipStream_t s_;
    NetLayer L_[kLayers];
    long long nparam_ = 0, nwb_ = 0;
    int adam_t_ = 0;
    // parameters
    float *P_ = nullptr, *G_ = nullptr, *M_ = nullptr, *V_ = nullptr;
    uint16_t *Wb_ = nullptr, *Wt_ = nullptr;
    uint16_t* Wf_ = nullptr;       // fragment-ordered weights of the forward kernels
    long long wf_off_[kLayers] = {};
    // activations (channels-last BF16)
    uint16_t *X_ = nullptr, *C1_ = nullptr, *D1_ = nullptr, *Q1_ = nullptr, *C2_ = nullptr, *D2_ = nullptr,
             *Q2_ = nullptr, *E3_ = nullptr;
    float* Y_ = nullptr;
    // backward
    uint16_t *gY_ = nullptr, *gD1_ = nullptr, *gD2_ = nullptr, *gE3_ = nullptr, *gE2_ = nullptr, *gE1_ = nullptr;
    float *dD1_ = nullptr, *dC1_ = nullptr, *dC2_ = nullptr, *dQ2_ = nullptr, *dQ1_ = nullptr;
    float* wpart_ = nullptr;
    long long wpart_floats_ = 0;
    double* red_ = nullptr;  // reduction partials
    double* sc_ = nullptr;   // device scalars: [0] mean p_prev, [1] s_r, [2] loss, [3] s_p
};

}  // namespace stp

/*
 * Oracle, part 4: the small MLP of the learned smoother (8 -> 64 -> 64 -> 4,
 * tanh hidden layers), forward pass, loss and its exact gradient by the chain
 * rule, in FP64 from the same BF16 weights.  TEST INFRASTRUCTURE ONLY (see
 * oracle.h).  Parameter order: W1[64][8] b1[64] W2[64][64] b2[64] W3[4][64] b3[4].
 * Loss: mean over samples and the 4 outputs of the squared error.
 * Pins: central finite differences of the loss (tests/test_oracle_mlp.py).
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { NI = 8, NH = 64, NO = 4 };
#define OW1 0
#define OB1 (OW1 + NH * NI)
#define OW2 (OB1 + NH)
#define OB2 (OW2 + NH * NH)
#define OW3 (OB2 + NH)
#define OB3 (OW3 + NO * NH)
#define NP (OB3 + NO)

int or_mlp_nparam(void) { return NP; }

/* a BF16 bit pattern is the upper half of an FP32 */
double or_bf16_value(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, sizeof f);
    return (double)f;
}

static void weights(const uint16_t *wb, double *w)
{
    for (int k = 0; k < NP; k++) w[k] = or_bf16_value(wb[k]);
}

static void forward1(const double *w, const double *x, double *h1, double *h2, double *y)
{
    for (int i = 0; i < NH; i++) {
        double a = w[OB1 + i];
        for (int j = 0; j < NI; j++) a += w[OW1 + i * NI + j] * x[j];
        h1[i] = tanh(a);
    }
    for (int i = 0; i < NH; i++) {
        double a = w[OB2 + i];
        for (int j = 0; j < NH; j++) a += w[OW2 + i * NH + j] * h1[j];
        h2[i] = tanh(a);
    }
    for (int i = 0; i < NO; i++) {
        double a = w[OB3 + i];
        for (int j = 0; j < NH; j++) a += w[OW3 + i * NH + j] * h2[j];
        y[i] = a;
    }
}

void or_mlp_forward(const uint16_t *wb, const double *X, int B, double *Y)
{
    double *w = malloc(sizeof(double) * NP), h1[NH], h2[NH];
    weights(wb, w);
    for (int s = 0; s < B; s++) forward1(w, X + s * NI, h1, h2, Y + s * NO);
    free(w);
}

/* Loss and gradient with respect to the (BF16-valued) parameters, as doubles. */
double or_mlp_loss_grad_w(const double *w, const double *X, const double *T, int B, double *grad)
{
    double h1[NH], h2[NH], y[NO], dy[NO], d2[NH], d1[NH];
    if (grad) memset(grad, 0, sizeof(double) * NP);
    double loss = 0.0;
    for (int s = 0; s < B; s++) {
        const double *x = X + s * NI;
        forward1(w, x, h1, h2, y);
        for (int i = 0; i < NO; i++) {
            double e = y[i] - T[s * NO + i];
            loss += e * e;
            dy[i] = 2.0 * e / (NO * B);
        }
        if (!grad) continue;
        for (int j = 0; j < NH; j++) {
            double a = 0.0;
            for (int i = 0; i < NO; i++) a += w[OW3 + i * NH + j] * dy[i];
            d2[j] = a * (1.0 - h2[j] * h2[j]);
        }
        for (int j = 0; j < NH; j++) {
            double a = 0.0;
            for (int i = 0; i < NH; i++) a += w[OW2 + i * NH + j] * d2[i];
            d1[j] = a * (1.0 - h1[j] * h1[j]);
        }
        for (int i = 0; i < NO; i++) {
            grad[OB3 + i] += dy[i];
            for (int j = 0; j < NH; j++) grad[OW3 + i * NH + j] += dy[i] * h2[j];
        }
        for (int i = 0; i < NH; i++) {
            grad[OB2 + i] += d2[i];
            for (int j = 0; j < NH; j++) grad[OW2 + i * NH + j] += d2[i] * h1[j];
            grad[OB1 + i] += d1[i];
            for (int j = 0; j < NI; j++) grad[OW1 + i * NI + j] += d1[i] * x[j];
        }
    }
    return loss / (NO * B);
}

double or_mlp_loss_grad(const uint16_t *wb, const double *X, const double *T, int B, double *grad)
{
    double *w = malloc(sizeof(double) * NP);
    weights(wb, w);
    double l = or_mlp_loss_grad_w(w, X, T, B, grad);
    free(w);
    return l;
}
